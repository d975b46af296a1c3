// Create-time kernels: sorted string index, binary-search lookup, excitation
// lists with popcount phases and wavefront ballot compaction, same-spin
// operator values, and the determinant diagonal.
//
// Paper: arXiv 2503.10335, Sec. II.C (membership of an excited string in the
// selected set by a sorted index and binary search; single/double excitation
// link tables built once over the selected strings and reused by every
// matrix-vector product; the Slater-Condon rule and the [a,b] categories;
// the stored [0,0] diagonal) and Sec. III.C (link-table entry: target index,
// two orbital indices, a sign).
#include <vector>

#include "tbsci_internal.hpp"

namespace tbsci {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int nth_bit(uint64_t x, int n) {
    for (int k = 0; k < n; ++k) x &= x - 1;
    return __builtin_ctzll(x);
}

// bits set in mask below this lane (the ballot compaction offset)
__device__ __forceinline__ uint32_t lane_prefix(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int32_t find_str(const uint64_t *__restrict__ keys,
                                            const int32_t *__restrict__ pos, int64_t l,
                                            uint64_t s) {
    int64_t lo = 0, n = l;
    while (n > 0) {
        const int64_t half = n >> 1;
        if (keys[lo + half] < s) {
            lo += half + 1;
            n -= half + 1;
        } else {
            n = half;
        }
    }
    return (lo < l && keys[lo] == s) ? pos[lo] : -1;
}

// (x, y), x < y, of the t-th pair of n items in lexicographic order
__device__ __forceinline__ void pair_decode(int t, int n, int &x, int &y) {
    x = 0;
    while (t >= n - 1 - x) {
        t -= n - 1 - x;
        ++x;
    }
    y = x + 1 + t;
}

__device__ __forceinline__ uint64_t below(int k) { return (1ull << k) - 1ull; }

// Rank sort of unique keys: the rank of a key is the number of smaller keys.
__global__ __launch_bounds__(kBlock) void k_rank_sort(const uint64_t *__restrict__ str, int64_t l,
                                                      uint64_t *__restrict__ keys,
                                                      int32_t *__restrict__ pos) {
    __shared__ uint64_t tile[kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t mine = i < l ? str[i] : 0ull;
    int64_t rank = 0;
    for (int64_t t0 = 0; t0 < l; t0 += kBlock) {
        const int64_t t = t0 + threadIdx.x;
        tile[threadIdx.x] = t < l ? str[t] : ~0ull;
        __syncthreads();
        const int n = (int)(l - t0 < kBlock ? l - t0 : kBlock);
        for (int k = 0; k < n; ++k) rank += (tile[k] < mine);
        __syncthreads();
    }
    if (i < l) {
        keys[rank] = mine;
        pos[rank] = (int32_t)i;
    }
}

__global__ void k_lookup(const uint64_t *__restrict__ keys, const int32_t *__restrict__ pos,
                         int64_t l, const uint64_t *__restrict__ q, int64_t n,
                         int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = find_str(keys, pos, l, q[i]);
}

// Single excitations of row I (one wavefront per row).  Candidates are
// enumerated as (p, q): p = the occupied orbital of I removed, q = 0..M-1
// added; q == p is the occupation entry, q in I otherwise is not a
// candidate.  Candidate order is (p, q), so compaction by ballot keeps the
// canonical order.
template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_singles(const uint64_t *__restrict__ str, int64_t l,
                                                    int M, const uint64_t *__restrict__ keys,
                                                    const int32_t *__restrict__ pos,
                                                    int64_t *__restrict__ cnt,
                                                    const int64_t *__restrict__ ptr,
                                                    Ent *__restrict__ ent) {
    const int lane = threadIdx.x & 63;
    const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    if (row >= l) return;  // uniform per wavefront
    const uint64_t I = str[row];
    const int n = __popcll(I);
    const int ncand = n * M;
    const int64_t base = FILL ? ptr[row] : 0;
    int64_t count = 0;
    for (int c0 = 0; c0 < ncand; c0 += 64) {
        const int c = c0 + lane;
        bool ok = false;
        Ent e{-1, 0u};
        if (c < ncand) {
            const int p = nth_bit(I, c / M), q = c % M;
            if (q == p) {
                ok = true;
                e.j = (int32_t)row;
                e.o = (uint32_t)(p | (q << 6) | (fold_pair(p, q) << 16));
            } else if (!((I >> q) & 1ull)) {
                const uint64_t J = I ^ (1ull << p) ^ (1ull << q);
                const int32_t j = find_str(keys, pos, l, J);
                if (j >= 0) {
                    const int lo = p < q ? p : q, hi = p < q ? q : p;
                    const uint64_t between = below(hi) & ~((2ull << lo) - 1ull);
                    const uint32_t neg = (uint32_t)(__popcll(I & between) & 1);
                    ok = true;
                    e.j = j;
                    e.o = (uint32_t)(p | (q << 6)) | (neg << 12) | ((uint32_t)fold_pair(p, q) << 16);
                }
            }
        }
        const uint64_t m = __ballot(ok);
        if (FILL && ok) ent[base + count + lane_prefix(m)] = e;
        count += __popcll(m);
    }
    if (!FILL && lane == 0) cnt[row] = count;
}

// Double excitations of row I: remove i < jj (occupied in I), add a < b
// (empty in I); order (i, jj, a, b).  The sign is <I| a+_i a+_jj a_b a_a |J>,
// obtained as the phase of a+_a a+_b a_jj a_i applied to I one operator at
// a time (each operator contributes (-1)^(occupied orbitals below it)).
template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_doubles(const uint64_t *__restrict__ str, int64_t l,
                                                    int M, const uint64_t *__restrict__ keys,
                                                    const int32_t *__restrict__ pos,
                                                    int64_t *__restrict__ cnt,
                                                    const int64_t *__restrict__ ptr,
                                                    Ent *__restrict__ ent) {
    const int lane = threadIdx.x & 63;
    const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    if (row >= l) return;
    const uint64_t I = str[row];
    const uint64_t full = M == 64 ? ~0ull : below(M);
    const uint64_t V = ~I & full;
    const int n = __popcll(I), nv = M - n;
    const int no2 = n * (n - 1) / 2, nv2 = nv * (nv - 1) / 2;
    const int64_t ncand = (int64_t)no2 * nv2;
    const int64_t base = FILL ? ptr[row] : 0;
    int64_t count = 0;
    for (int64_t c0 = 0; c0 < ncand; c0 += 64) {
        const int64_t c = c0 + lane;
        bool ok = false;
        Ent e{-1, 0u};
        if (c < ncand) {
            int x, y, u, v;
            pair_decode((int)(c / nv2), n, x, y);
            pair_decode((int)(c % nv2), nv, u, v);
            const int i = nth_bit(I, x), jj = nth_bit(I, y), a = nth_bit(V, u), b = nth_bit(V, v);
            const uint64_t J = I ^ (1ull << i) ^ (1ull << jj) ^ (1ull << a) ^ (1ull << b);
            const int32_t j = find_str(keys, pos, l, J);
            if (j >= 0) {
                uint64_t s = I;
                int neg = __popcll(s & below(i));
                s ^= 1ull << i;
                neg += __popcll(s & below(jj));
                s ^= 1ull << jj;
                neg += __popcll(s & below(b));
                s ^= 1ull << b;
                neg += __popcll(s & below(a));
                ok = true;
                e.j = j;
                e.o = (uint32_t)(i | (jj << 6) | (a << 12) | (b << 18)) | ((uint32_t)(neg & 1) << 24);
            }
        }
        const uint64_t m = __ballot(ok);
        if (FILL && ok) ent[base + count + lane_prefix(m)] = e;
        count += __popcll(m);
    }
    if (!FILL && lane == 0) cnt[row] = count;
}

// Exclusive scan of n counts into ptr[0..n] (ptr[n] = total), one block.
__global__ __launch_bounds__(1024) void k_scan(const int64_t *__restrict__ cnt, int64_t n,
                                               int64_t *__restrict__ ptr) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t b = t * chunk, e = b + chunk < n ? b + chunk : n;
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += cnt[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = t ? part[t - 1] : 0;
    for (int64_t i = b; i < e; ++i) {
        ptr[i] = run;
        run += cnt[i];
    }
    if (t == 1023) ptr[n] = part[1023];
}

__device__ __forceinline__ double g4(const double *__restrict__ eri, int M, int p, int q, int r,
                                     int s) {
    return eri[(((int64_t)p * M + q) * M + r) * M + s];
}

// Same-spin diagonal d(I) = sum_i h_ii + 1/2 sum_{i,j in I} [(ii|jj) - (ij|ji)]
// and jocc[I][p] = sum_{r in I} (pp|rr).
__global__ void k_spin_diag(const uint64_t *__restrict__ str, int64_t l, int M,
                            const double *__restrict__ h, const double *__restrict__ eri,
                            double *__restrict__ dsame, double *__restrict__ jocc) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= l) return;
    const uint64_t I = str[row];
    double one = 0.0, two = 0.0;
    for (uint64_t x = I; x; x &= x - 1) {
        const int i = __builtin_ctzll(x);
        one += h[i * M + i];
        for (uint64_t y = I; y; y &= y - 1) {
            const int j = __builtin_ctzll(y);
            two += g4(eri, M, i, i, j, j) - g4(eri, M, i, j, j, i);
        }
    }
    dsame[row] = one + 0.5 * two;
    for (int p = 0; p < M; ++p) {
        double s = 0.0;
        for (uint64_t y = I; y; y &= y - 1) {
            const int r = __builtin_ctzll(y);
            s += g4(eri, M, p, p, r, r);
        }
        jocc[row * M + p] = s;
    }
}

__global__ void k_a_ptr(const int64_t *__restrict__ s_ptr, const int64_t *__restrict__ d_ptr,
                        int64_t l, int n, int64_t *__restrict__ a_ptr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= l) a_ptr[i] = i + (s_ptr[i] - (int64_t)n * i) + d_ptr[i];
}

// Same-spin operator row I (one wavefront per row): diagonal, then singles
// (p != q) in list order, then doubles in list order.
//  single (remove p from I, add q):   s [h_pq + sum_{k in I} ((pq|kk) - (pk|kq))]
//  double (remove i<jj, add a<b):     s [(ia|jj b) - (ib|jj a)]
__global__ __launch_bounds__(kBlock) void k_same_spin(
    const uint64_t *__restrict__ str, int64_t l, int M, const double *__restrict__ h,
    const double *__restrict__ eri, const int64_t *__restrict__ s_ptr,
    const Ent *__restrict__ s_ent, const int64_t *__restrict__ d_ptr,
    const Ent *__restrict__ d_ent, const double *__restrict__ dsame,
    const int64_t *__restrict__ a_ptr, int32_t *__restrict__ a_col, double *__restrict__ a_val,
    float *__restrict__ a_val32) {
    const int lane = threadIdx.x & 63;
    const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    if (row >= l) return;
    const uint64_t I = str[row];
    const int64_t base = a_ptr[row];
    if (lane == 0) {
        a_col[base] = (int32_t)row;
        a_val[base] = dsame[row];
        a_val32[base] = (float)dsame[row];
    }
    int64_t count = 1;
    const int64_t sb = s_ptr[row], se = s_ptr[row + 1];
    for (int64_t e0 = sb; e0 < se; e0 += 64) {
        const int64_t e = e0 + lane;
        bool ok = false;
        double v = 0.0;
        int32_t j = -1;
        if (e < se) {
            const Ent en = s_ent[e];
            const int p = en.o & 63, q = (en.o >> 6) & 63;
            if (p != q) {
                ok = true;
                j = en.j;
                double t = h[p * M + q];
                for (uint64_t x = I; x; x &= x - 1) {
                    const int k = __builtin_ctzll(x);
                    t += g4(eri, M, p, q, k, k) - g4(eri, M, p, k, k, q);
                }
                v = ((en.o >> 12) & 1) ? -t : t;
            }
        }
        const uint64_t m = __ballot(ok);
        if (ok) {
            const int64_t at = base + count + lane_prefix(m);
            a_col[at] = j;
            a_val[at] = v;
            a_val32[at] = (float)v;
        }
        count += __popcll(m);
    }
    const int64_t db = d_ptr[row], de = d_ptr[row + 1];
    for (int64_t e = db + lane; e < de; e += 64) {
        const Ent en = d_ent[e];
        const int i = en.o & 63, jj = (en.o >> 6) & 63, a = (en.o >> 12) & 63, b = (en.o >> 18) & 63;
        const double t = g4(eri, M, i, a, jj, b) - g4(eri, M, i, b, jj, a);
        const double v = ((en.o >> 24) & 1) ? -t : t;
        const int64_t at = base + count + (e - db);
        a_col[at] = en.j;
        a_val[at] = v;
        a_val32[at] = (float)v;
    }
}

// Regroup each singles row by (MFMA tile t = pair / 16, lane group
// g = (pair % 16) & 3) of the folded pair index: a counting sort per row, one
// thread per row, list order kept inside a group.  Group key = 4 t + g.
__global__ void k_group_by_tile(const int64_t *__restrict__ s_ptr, const Ent *__restrict__ s_ent,
                                int64_t l, int ngroup, Ent *__restrict__ g_ent,
                                int32_t *__restrict__ g_off) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= l) return;
    const int64_t b = s_ptr[row], e = s_ptr[row + 1];
    int32_t *off = g_off + row * (ngroup + 1);
    auto key = [](uint32_t o) {
        const int pair = (int)(o >> 16);
        return 4 * (pair >> 4) + ((pair & 15) & 3);
    };
    for (int t = 0; t <= ngroup; ++t) off[t] = 0;
    for (int64_t i = b; i < e; ++i) off[key(s_ent[i].o) + 1]++;
    for (int t = 0; t < ngroup; ++t) off[t + 1] += off[t];
    for (int t = ngroup; t > 0; --t) off[t] = off[t - 1];  // off[t + 1] = start of group t
    off[0] = 0;
    for (int64_t i = b; i < e; ++i) g_ent[b + off[key(s_ent[i].o) + 1]++] = s_ent[i];
    // off[t + 1] advanced to the end of group t = start of group t + 1
}

// Same-spin rows regrouped by source chunk (col / chunk), stable within a
// chunk; off[row (nch + 1) + c] = start of chunk c relative to the row.
__global__ void k_chunk_rows(const int64_t *__restrict__ a_ptr, const int32_t *__restrict__ a_col,
                             const double *__restrict__ a_val, const float *__restrict__ a_val32,
                             int64_t l, int nch, int64_t chunk, int32_t *__restrict__ off,
                             int32_t *__restrict__ b_col, double *__restrict__ b_val,
                             float *__restrict__ b_val32) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= l) return;
    const int64_t b = a_ptr[row], e = a_ptr[row + 1];
    int32_t *o = off + row * (nch + 1);
    for (int c = 0; c <= nch; ++c) o[c] = 0;
    for (int64_t i = b; i < e; ++i) o[a_col[i] / chunk + 1]++;
    for (int c = 0; c < nch; ++c) o[c + 1] += o[c];
    // o[c] = start of chunk c; place with running cursors kept in o[c], then
    // shift back
    for (int64_t i = b; i < e; ++i) {
        const int c = (int)(a_col[i] / chunk);
        const int64_t at = b + o[c]++;
        b_col[at] = a_col[i];
        b_val[at] = a_val[i];
        b_val32[at] = a_val32[i];
    }
    for (int c = nch; c > 0; --c) o[c] = o[c - 1];
    o[0] = 0;
}

// H_KK = d_alpha(I) + d_beta(I') + sum_{p in I} jocc_beta[I'][p]
__global__ void k_full_diag(const uint64_t *__restrict__ astr, int64_t la, int64_t lb, int M,
                            const double *__restrict__ da, const double *__restrict__ db,
                            const double *__restrict__ jb, double *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= la * lb) return;
    const int64_t ia = k / lb, ib = k - ia * lb;
    double v = da[ia] + db[ib];
    const double *jr = jb + ib * M;
    for (uint64_t x = astr[ia]; x; x &= x - 1) v += jr[__builtin_ctzll(x)];
    out[k] = v;
}


template <typename T>
T *dalloc(size_t n) {
    void *p = nullptr;
    if (n == 0) n = 1;
    TB_HIP(hipMalloc(&p, n * sizeof(T)));
    return (T *)p;
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

void build_spin(Ctx &c, Spin &s, const uint64_t *host_str, hipStream_t st) {
    const int64_t l = s.l;
    const int M = c.M;
    s.str = dalloc<uint64_t>(l);
    s.keys = dalloc<uint64_t>(l);
    s.pos = dalloc<int32_t>(l);
    TB_HIP(hipMemcpyAsync(s.str, host_str, l * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    k_rank_sort<<<blocks_for(l, kBlock), kBlock, 0, st>>>(s.str, l, s.keys, s.pos);
    TB_HIP(hipGetLastError());

    int64_t *cnt = dalloc<int64_t>(l);
    const unsigned wblocks = blocks_for(l, kBlock / 64);
    // singles (with occupation entries)
    s.s_ptr = dalloc<int64_t>(l + 1);
    k_singles<false><<<wblocks, kBlock, 0, st>>>(s.str, l, M, s.keys, s.pos, cnt, nullptr, nullptr);
    k_scan<<<1, 1024, 0, st>>>(cnt, l, s.s_ptr);
    TB_HIP(hipGetLastError());
    std::vector<int64_t> hp(l + 1);
    TB_HIP(hipMemcpyAsync(hp.data(), s.s_ptr, (l + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TB_HIP(hipStreamSynchronize(st));
    s.n_s = hp[l];
    s.max_s = 0;
    for (int64_t i = 0; i < l; ++i) s.max_s = std::max<int64_t>(s.max_s, hp[i + 1] - hp[i]);
    s.s_ent = dalloc<Ent>(s.n_s);
    k_singles<true><<<wblocks, kBlock, 0, st>>>(s.str, l, M, s.keys, s.pos, nullptr, s.s_ptr, s.s_ent);
    TB_HIP(hipGetLastError());
    // singles regrouped by MFMA pair tile (the opposite-spin scatter reads these)
    {
        const int ngroup = 4 * ((c.P + 15) / 16);
        s.g_ent = dalloc<Ent>(s.n_s);
        s.g_off = dalloc<int32_t>((size_t)l * (ngroup + 1));
        k_group_by_tile<<<blocks_for(l, 128), 128, 0, st>>>(s.s_ptr, s.s_ent, l, ngroup, s.g_ent,
                                                             s.g_off);
        TB_HIP(hipGetLastError());
    }
    // doubles
    s.d_ptr = dalloc<int64_t>(l + 1);
    k_doubles<false><<<wblocks, kBlock, 0, st>>>(s.str, l, M, s.keys, s.pos, cnt, nullptr, nullptr);
    k_scan<<<1, 1024, 0, st>>>(cnt, l, s.d_ptr);
    TB_HIP(hipGetLastError());
    TB_HIP(hipMemcpyAsync(&s.n_d, s.d_ptr + l, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TB_HIP(hipStreamSynchronize(st));
    s.d_ent = dalloc<Ent>(s.n_d);
    k_doubles<true><<<wblocks, kBlock, 0, st>>>(s.str, l, M, s.keys, s.pos, nullptr, s.d_ptr, s.d_ent);
    TB_HIP(hipGetLastError());
    // same-spin diagonal and Coulomb occupation sums
    s.dsame = dalloc<double>(l);
    s.jocc = dalloc<double>((size_t)l * M);
    k_spin_diag<<<blocks_for(l, 128), 128, 0, st>>>(s.str, l, M, c.h, c.eri, s.dsame, s.jocc);
    // same-spin operator CSR
    s.a_ptr = dalloc<int64_t>(l + 1);
    k_a_ptr<<<blocks_for(l + 1, kBlock), kBlock, 0, st>>>(s.s_ptr, s.d_ptr, l, s.n, s.a_ptr);
    s.n_a = l + (s.n_s - (int64_t)s.n * l) + s.n_d;
    s.a_col = dalloc<int32_t>(s.n_a);
    s.a_val = dalloc<double>(s.n_a);
    s.a_val32 = dalloc<float>(s.n_a);
    k_same_spin<<<wblocks, kBlock, 0, st>>>(s.str, l, M, c.h, c.eri, s.s_ptr, s.s_ent, s.d_ptr,
                                             s.d_ent, s.dsame, s.a_ptr, s.a_col, s.a_val, s.a_val32);
    TB_HIP(hipGetLastError());
    s.chunk = sweep_chunk(l, s.n_a);
    s.nch = s.chunk ? (int)((l + s.chunk - 1) / s.chunk) : 1;
    if (s.nch > 1) {
        s.b_off = dalloc<int32_t>((size_t)l * (s.nch + 1));
        s.b_col = dalloc<int32_t>(s.n_a);
        s.b_val = dalloc<double>(s.n_a);
        s.b_val32 = dalloc<float>(s.n_a);
        k_chunk_rows<<<blocks_for(l, 128), 128, 0, st>>>(s.a_ptr, s.a_col, s.a_val, s.a_val32, l,
                                                          s.nch, s.chunk, s.b_off, s.b_col,
                                                          s.b_val, s.b_val32);
        TB_HIP(hipGetLastError());
    }
    TB_HIP(hipStreamSynchronize(st));
    TB_HIP(hipFree(cnt));
}

namespace {

// entries of each same-spin row that are kept: the diagonal (first) and
// every element that is not exactly zero
__global__ void k_nz_count(const int64_t *__restrict__ a_ptr, const double *__restrict__ a_val,
                           int64_t l, int64_t *__restrict__ cnt) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= l) return;
    int64_t n = 0;
    for (int64_t i = a_ptr[row]; i < a_ptr[row + 1]; ++i)
        n += (i == a_ptr[row] || a_val[i] != 0.0) ? 1 : 0;
    cnt[row] = n;
}

__global__ void k_nz_copy(const int64_t *__restrict__ a_ptr, const int32_t *__restrict__ a_col,
                          const double *__restrict__ a_val, const float *__restrict__ a_val32,
                          int64_t l, const int64_t *__restrict__ n_ptr, int32_t *__restrict__ n_col,
                          double *__restrict__ n_val, float *__restrict__ n_val32) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= l) return;
    int64_t o = n_ptr[row];
    for (int64_t i = a_ptr[row]; i < a_ptr[row + 1]; ++i)
        if (i == a_ptr[row] || a_val[i] != 0.0) {
            n_col[o] = a_col[i];
            n_val[o] = a_val[i];
            n_val32[o] = a_val32[i];
            ++o;
        }
}

}  // namespace

void compact_same_spin(Ctx &c, Spin &s, hipStream_t st) {
    (void)c;
    const int64_t l = s.l;
    int64_t *cnt = dalloc<int64_t>(l);
    int64_t *np = dalloc<int64_t>(l + 1);
    k_nz_count<<<blocks_for(l, 128), 128, 0, st>>>(s.a_ptr, s.a_val, l, cnt);
    k_scan<<<1, 1024, 0, st>>>(cnt, l, np);
    TB_HIP(hipGetLastError());
    int64_t n = 0;
    TB_HIP(hipMemcpyAsync(&n, np + l, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TB_HIP(hipStreamSynchronize(st));
    int32_t *ncol = dalloc<int32_t>(n);
    double *nval = dalloc<double>(n);
    float *nval32 = dalloc<float>(n);
    k_nz_copy<<<blocks_for(l, 128), 128, 0, st>>>(s.a_ptr, s.a_col, s.a_val, s.a_val32, l, np,
                                                   ncol, nval, nval32);
    TB_HIP(hipGetLastError());
    TB_HIP(hipStreamSynchronize(st));
    void *old[] = {s.a_ptr, s.a_col, s.a_val, s.a_val32, s.b_off, s.b_col, s.b_val, s.b_val32, cnt};
    for (void *p : old)
        if (p) TB_HIP(hipFree(p));
    s.a_ptr = np;
    s.a_col = ncol;
    s.a_val = nval;
    s.a_val32 = nval32;
    s.b_off = nullptr;
    s.b_col = nullptr;
    s.b_val = nullptr;
    s.b_val32 = nullptr;
    s.n_a = n;
    s.chunk = sweep_chunk(l, s.n_a);
    s.nch = s.chunk ? (int)((l + s.chunk - 1) / s.chunk) : 1;
    if (s.nch > 1) {
        s.b_off = dalloc<int32_t>((size_t)l * (s.nch + 1));
        s.b_col = dalloc<int32_t>(s.n_a);
        s.b_val = dalloc<double>(s.n_a);
        s.b_val32 = dalloc<float>(s.n_a);
        k_chunk_rows<<<blocks_for(l, 128), 128, 0, st>>>(s.a_ptr, s.a_col, s.a_val, s.a_val32, l,
                                                          s.nch, s.chunk, s.b_off, s.b_col,
                                                          s.b_val, s.b_val32);
        TB_HIP(hipGetLastError());
        TB_HIP(hipStreamSynchronize(st));
    }
}

void launch_lookup(const Spin &s, const uint64_t *q, int64_t n, int32_t *out, hipStream_t st) {
    if (n <= 0) return;
    k_lookup<<<blocks_for(n, kBlock), kBlock, 0, st>>>(s.keys, s.pos, s.l, q, n, out);
    TB_HIP(hipGetLastError());
}

void launch_full_diag(const Ctx &c, double *out, hipStream_t st) {
    const int64_t n = c.sp[0].l * c.sp[1].l;
    k_full_diag<<<blocks_for(n, kBlock), kBlock, 0, st>>>(c.sp[0].str, c.sp[0].l, c.sp[1].l, c.M,
                                                          c.sp[0].dsame, c.sp[1].dsame,
                                                          c.sp[1].jocc, out);
    TB_HIP(hipGetLastError());
}


void build_ks_classes(Spin &s) {
    if (s.ks_rows) TB_HIP(hipFree(s.ks_rows));
    s.ks_rows = nullptr;
    std::vector<int64_t> ptr((size_t)s.l + 1);
    TB_HIP(hipMemcpy(ptr.data(), s.s_ptr, ptr.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    static const int kcls[5] = {8, 16, 24, 28, 32};
    std::vector<int32_t> cls[5];
    for (int64_t i = 0; i < s.l; ++i) {
        const int64_t ks = (ptr[(size_t)i + 1] - ptr[(size_t)i] + 3) / 4;
        int k = 0;
        while (k < 4 && ks > kcls[k]) ++k;
        cls[k].push_back((int32_t)i);
    }
    std::vector<int32_t> rows;
    rows.reserve((size_t)s.l);
    s.ks_off[0] = 0;
    for (int k = 0; k < 5; ++k) {
        rows.insert(rows.end(), cls[k].begin(), cls[k].end());
        s.ks_off[k + 1] = (int64_t)rows.size();
    }
    TB_HIP(hipMalloc((void **)&s.ks_rows, std::max<size_t>(rows.size(), 1) * sizeof(int32_t)));
    if (!rows.empty())
        TB_HIP(hipMemcpy(s.ks_rows, rows.data(), rows.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice));
}

}  // namespace tbsci
