// Same-spin term of sigma in hole-pair form (Sec. II.C, the [2,0] / [0,2]
// categories with the same-spin parts of [1,0], [0,1] and [0,0]).
//
// On n-electron strings of one spin (n >= 2) the spin's whole same-spin
// Hamiltonian, one-body part included, is
//
//   H_s = sum_{p<r} sum_{q<s} W[pr][qs] a+_p a+_r a_s a_q
//   W[pr][qs] = (pq|rs) - (ps|rq)
//             + (h_pq d_rs + h_rs d_pq - h_ps d_rq - h_rq d_ps) / (n - 1)
//
// (the two-body sum over ordered pairs; the one-body part through
// a+_p a_q = a+_p N a_q / (n - 1), N counting the n - 1 electrons left
// after a_q).  Resolving the identity on the (n-2)-electron strings K
// between the creators and the annihilators:
//
//   (A_s X)[I][c] = sum_{K in I} s(I; K) sum_{J contains K}
//                       W[pair(I - K)][pair(J - K)] s(J; K) X[J][c]
//
// with s(Z; K) = <K| a_y a_x |Z> for Z = K + {x < y}.  So for each hole
// string K: gather the rows of X of the strings J that contain K (signed),
// multiply them by the dense block of W of their pairs (MFMA, k_hole_gemm),
// and every string I that contains K reads its row of that product back
// (k_hole_sum: the n(n-1)/2 hole strings of I, summed in a fixed order, no
// atomics).  I and J both run over the spin's strings only, so the
// projection onto the selected strings is exact.  The products of one
// window of columns pass through a buffer in HBM.

#include <algorithm>
#include <vector>

#include "tbsci_internal.hpp"

namespace tbsci {
namespace {

constexpr int kHB = 256;               // threads per block, both kernels
constexpr int kHoleMax = 128;          // longest hole-string list taken
constexpr size_t kHoleWorkCap = size_t(4) << 30;

inline int pair_id(int p, int q) { return q * (q - 1) / 2 + p; }  // p < q

template <typename T>
struct HoleMma;
// Operands of the 16x16x4 MFMAs (lane l): A[m][k] with m = l%16, k = l/16;
// B[k][n] with k = l/16, n = l%16; accumulator register r holds
// D[row(l, r)][l%16]
template <>
struct HoleMma<double> {
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct HoleMma<float> {
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// Barrier for the LDS staging: waits for this wave's LDS operations only
// (lgkmcnt), not for its global loads in flight or its stores of products,
// which a full __syncthreads would also drain
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <typename T>
struct Vec16;  // 16-byte vector of T
template <>
struct Vec16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};

// Products of one hole string K (block K / nb) over the window columns
// [cb0, cb0 + cpb) (block K % nb):
//   Y[e][c] = sum_{e'} W[pair e][pair e'] s_e' X[x_e'][c0 + c]
// for the entries e, e' of K (e global entry positions, Y row stride ldy).
// Wave w takes M-tiles w, w + 4, ... (16 entries each) with its A fragments
// in registers for the whole block.  The signed X rows of K are staged in
// LDS 16 CT columns at a time, all 4 KS rows (rows past the list zero), in
// loads of VL elements (16 bytes when the rows are 16-byte aligned); the
// loads of the next tile are issued before the MFMAs of the current one
// and applied (sign, zero) when stored, so nothing waits for them early.
// The k loop runs all KS steps (A is zero past the list), without branches.
// KS >= ceil(longest list / 4); MTW = 1 for lists of up to 64 entries
// (four M-tiles), 2 for up to 128.
template <typename T, int KS, int MTW, int CT, int VL>
__global__ __launch_bounds__(kHB) void k_hole_gemm(int64_t nb, int64_t cpb, int64_t nwin,
                                                  int64_t ldx, int64_t c0, int64_t ldy,
                                                  const int64_t *__restrict__ hptr,
                                                  const uint2 *__restrict__ hent,
                                                  const T *__restrict__ W, int pp,
                                                  const T *__restrict__ X, T *__restrict__ Y) {
    using M = HoleMma<T>;
    constexpr int VEC = 16 / sizeof(T);  // elements per thread and staged row segment
    constexpr int NL = VEC / VL;         // loads per segment
    constexpr int TW = 16 * CT;          // columns per staged tile
    constexpr int LD = TW + VEC;         // padded LDS row (16-byte aligned)
    constexpr int LPR = TW / VEC;        // threads per staged row
    constexpr int RPP = kHB / LPR;       // rows per staging pass
    constexpr int R = 4 * KS;            // staged rows
    constexpr int NP = (R + RPP - 1) / RPP;
    static_assert(kHB % LPR == 0 && NP * NL <= 32, "staging layout");
    typedef T TL __attribute__((ext_vector_type(VL)));
    __shared__ __align__(16) T xs[R * LD];
    __shared__ int64_t xoff[R];  // X row offset of staged row r, or -1
    __shared__ int xneg[R];
    const int64_t K = blockIdx.x / nb;
    const int64_t cb0 = (blockIdx.x - K * nb) * cpb;
    const int64_t cb1 = std::min(nwin, cb0 + cpb);
    const int64_t e0 = hptr[K];
    const int nK = (int)(hptr[K + 1] - e0);
    const int MT = (nK + 15) >> 4;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, cl = lane & 15;

    for (int r = tid; r < R; r += kHB) {
        int64_t o = -1;
        int neg = 0;
        if (r < nK) {
            const uint2 en = hent[e0 + r];
            o = (int64_t)en.x * ldx + c0;
            neg = (int)(en.y >> 16);
        }
        xoff[r] = o;
        xneg[r] = neg;
    }
    // A[m][k] = W[pair(16 mt + m)][pair(4 ks + k)], zero outside the list
    T a[MTW][KS];
#pragma unroll
    for (int w = 0; w < MTW; ++w) {
        const int er = 16 * (wave + 4 * w) + cl;
        const int64_t prow = er < nK ? (int64_t)(hent[e0 + er].y & 0xffffu) * pp : 0;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int ec = 4 * ks + g;
            T v = T(0);
            if (er < nK && ec < nK) v = W[prow + (hent[e0 + ec].y & 0xffffu)];
            a[w][ks] = v;
        }
    }
    __syncthreads();

    // this thread's staged segments: rows p RPP + sr, columns sc .. sc + VEC
    const int sr = tid / LPR, sc = (tid - sr * LPR) * VEC;
    TL buf[NP][NL];
    uint32_t valid = 0;  // bit p NL + k: segment part k of pass p is inside the list and window
    auto load = [&](int64_t cc) {
        valid = 0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int r = p * RPP + sr;
            const int64_t o = r < R ? xoff[r] : -1;
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const int64_t c = cc + sc + k * VL;
                const bool ok = o >= 0 && c + VL <= cb1;
                buf[p][k] = *(const TL *)(X + (ok ? o + c : 0));
                valid |= (uint32_t)ok << (p * NL + k);
            }
        }
    };
    load(cb0);
    for (int64_t cc = cb0; cc < cb1; cc += TW) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int r = p * RPP + sr;
            if (r < R) {
                const bool neg = xneg[r] != 0;
#pragma unroll
                for (int k = 0; k < NL; ++k) {
                    TL v = buf[p][k];
                    if (neg) v = -v;
                    if (!((valid >> (p * NL + k)) & 1u)) v = TL{};
                    *(TL *)(xs + r * LD + sc + k * VL) = v;
                }
            }
        }
        lds_barrier();
        if (cc + TW < cb1) load(cc + TW);  // in flight during the MFMAs
#pragma unroll
        for (int w = 0; w < MTW; ++w) {
            const int mt = wave + 4 * w;
            if (mt < MT) {
                typename M::acc_t acc[CT];
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) acc[ct] = typename M::acc_t{0, 0, 0, 0};
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                    for (int ct = 0; ct < CT; ++ct)
                        acc[ct] = M::mma(a[w][ks], xs[(4 * ks + g) * LD + 16 * ct + cl], acc[ct]);
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                    const int64_t col = cc + 16 * ct + cl;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int e = 16 * mt + M::row(lane, r);
                        if (e < nK && col < cb1)
                            __builtin_nontemporal_store(acc[ct][r], &Y[(e0 + e) * ldy + col]);
                    }
                }
            }
        }
        lds_barrier();  // every wave's reads of this tile done before the next staging
    }
}

// O[x][c0 + c] = sum_t s_t Y[e_t][c] over the npo entries e_t of string x
// (inv: e | sign << 31), in entry order.  tpr threads per string (a
// multiple of 64), VEC columns per thread with 16-byte loads of Y (its rows
// hold ldy >= nwin columns, ldy a multiple of 64).
template <typename T>
__global__ __launch_bounds__(kHB) void k_hole_sum(int64_t l, int tpr, int npo, int64_t nwin,
                                                 int64_t ldo, int64_t c0, int64_t ldy,
                                                 const uint32_t *__restrict__ inv,
                                                 const T *__restrict__ Y, T *__restrict__ O) {
    using TV = typename Vec16<T>::type;
    constexpr int VEC = 16 / sizeof(T);
    const int64_t x = (int64_t)blockIdx.x * (kHB / tpr) + threadIdx.x / tpr;
    if (x >= l) return;
    const uint32_t *iv = inv + x * npo;
    T *o = O + x * ldo + c0;
    for (int64_t c = (int64_t)(threadIdx.x % tpr) * VEC; c < nwin; c += (int64_t)tpr * VEC) {
        TV acc = {};
#pragma unroll 4
        for (int t = 0; t < npo; ++t) {
            const uint32_t u = iv[t];
            const TV v =
                __builtin_nontemporal_load((const TV *)(Y + (int64_t)(u & 0x7fffffffu) * ldy + c));
            acc += (u >> 31) ? -v : v;
        }
#pragma unroll
        for (int k = 0; k < VEC; ++k)
            if (c + k < nwin) o[c + k] = acc[k];
    }
}

template <typename T, int KS, int MTW, int CT, int VL>
void launch_gemm_t(const Spin &s, int64_t nb, int64_t cpb, int64_t nwin, int64_t ldx, int64_t c0,
                   int64_t ldy, const T *W, const T *X, T *Y, hipStream_t st) {
    k_hole_gemm<T, KS, MTW, CT, VL><<<(unsigned)(s.n_hole * nb), kHB, 0, st>>>(
        nb, cpb, nwin, ldx, c0, ldy, s.h_ptr, s.h_ent, W, s.pp, X, Y);
}

// k-step depth: the smallest instance that holds the longest list
template <typename T, int VL>
void launch_gemm_v(const Spin &s, int64_t nb, int64_t cpb, int64_t nwin, int64_t ldx, int64_t c0,
                   int64_t ldy, const T *W, const T *X, T *Y, hipStream_t st) {
    const int ks = (s.hmax + 3) / 4;
    if (ks <= 8)
        launch_gemm_t<T, 8, 1, 4, VL>(s, nb, cpb, nwin, ldx, c0, ldy, W, X, Y, st);
    else if (ks <= 12)
        launch_gemm_t<T, 12, 1, 4, VL>(s, nb, cpb, nwin, ldx, c0, ldy, W, X, Y, st);
    else if (ks <= 14)
        launch_gemm_t<T, 14, 1, 4, VL>(s, nb, cpb, nwin, ldx, c0, ldy, W, X, Y, st);
    else if (ks <= 16)
        launch_gemm_t<T, 16, 1, 4, VL>(s, nb, cpb, nwin, ldx, c0, ldy, W, X, Y, st);
    else if (ks <= 24)
        launch_gemm_t<T, 24, 2, 2, VL>(s, nb, cpb, nwin, ldx, c0, ldy, W, X, Y, st);
    else
        launch_gemm_t<T, 32, 2, 2, VL>(s, nb, cpb, nwin, ldx, c0, ldy, W, X, Y, st);
}

// 16-byte loads when every staged segment is 16-byte aligned (X aligned,
// its rows a whole number of 16-byte units long), else element loads
template <typename T>
void launch_gemm(const Spin &s, int64_t nb, int64_t cpb, int64_t nwin, int64_t ldx, int64_t c0,
                 int64_t ldy, const T *W, const T *X, T *Y, hipStream_t st) {
    constexpr int VEC = 16 / sizeof(T);
    if (ldx % VEC == 0 && (uintptr_t)X % 16 == 0)
        launch_gemm_v<T, VEC>(s, nb, cpb, nwin, ldx, c0, ldy, W, X, Y, st);
    else
        launch_gemm_v<T, 1>(s, nb, cpb, nwin, ldx, c0, ldy, W, X, Y, st);
}

template <typename T>
void hole_sweep_t(const Spin &s, int64_t ncols, const T *X, T *Y, void *work, size_t work_bytes,
                  hipStream_t st) {
    if (ncols == 0 || s.l == 0) return;
    // window: whole 64-column tiles whose products fit the buffer
    int64_t wn = (int64_t)(work_bytes / ((size_t)s.n_hent * sizeof(T))) / 64 * 64;
    wn = std::min(wn, (ncols + 63) / 64 * 64);
    if (wn < 64) throw Error(TBSCI_E_INVAL, "hole-pair sweep: product buffer too small");
    T *Yb = (T *)work;
    const T *W = sizeof(T) == 8 ? (const T *)(const void *)s.hW : (const T *)(const void *)s.hW32;
    const uint32_t *inv = (const uint32_t *)s.h_inv;
    constexpr int VEC = 16 / sizeof(T);
    for (int64_t c0 = 0; c0 < ncols; c0 += wn) {
        const int64_t nwin = std::min(wn, ncols - c0);
        // blocks of up to 512 columns: enough of them to fill the chip
        const int64_t cpb = std::min<int64_t>(512, (nwin + 63) / 64 * 64);
        const int64_t nb = (nwin + cpb - 1) / cpb;
        launch_gemm<T>(s, nb, cpb, nwin, ncols, c0, wn, W, X, Yb, st);
        TB_HIP(hipGetLastError());
        // threads per string: 64, 128 or 256, covering the window's vectors
        int tpr = 64;
        while (tpr < kHB && (int64_t)tpr * VEC < nwin) tpr *= 2;
        const int64_t rpb = kHB / tpr;
        k_hole_sum<T><<<(unsigned)((s.l + rpb - 1) / rpb), kHB, 0, st>>>(
            s.l, tpr, s.npo, nwin, ncols, c0, wn, inv, Yb, Y);
        TB_HIP(hipGetLastError());
    }
}

template <typename T>
T *upload(const std::vector<T> &v) {
    T *p = nullptr;
    TB_HIP(hipMalloc((void **)&p, std::max<size_t>(v.size(), 1) * sizeof(T)));
    if (!v.empty()) TB_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
}

}  // namespace

void free_hole(Spin &s) {
    void *ptrs[] = {s.h_ptr, s.h_ent, s.h_inv, s.hW, s.hW32};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    s.h_ptr = nullptr;
    s.h_ent = nullptr;
    s.h_inv = nullptr;
    s.hW = nullptr;
    s.hW32 = nullptr;
    s.hole = s.hole_auto = false;
    s.hole_mfma = 0.0;
    s.hmax = s.npo = s.pp = 0;
    s.n_hole = s.n_hent = 0;
}

// Build a spin's hole-pair index.  The automatic method takes a spin when
// its hole strings hold at least TBSCI_HOLE_AUTO_MIN strings on average
// (dense, FCI-like string sets: the product blocks are then large enough
// for the matrix cores) and the space is too large to share grouped
// launches (the beta sweep runs in blocks); without force the index is
// uploaded only for such a spin.
void hole_build(Ctx &c, int spin, bool force) {
    Spin &s = c.sp[spin];
    if (s.hole || (s.hole_built && !force)) return;
    s.hole_built = true;
    const int n = s.n, M = c.M;
    const int64_t l = s.l;
    if (n < 2 || l == 0) return;
    // the automatic method only takes spaces too large for grouped launches:
    // for the others nothing is built unless asked for
    const bool large = beta_block_rows(c.sp[0].l, c.sp[1].l, kWorkCap) < c.sp[0].l;
    if (!force && !large) return;
    std::vector<uint64_t> str((size_t)l);
    TB_HIP(hipMemcpy(str.data(), s.str, (size_t)l * 8, hipMemcpyDeviceToHost));
    const size_t M2 = (size_t)M * M;
    std::vector<double> h(M2), eri(M2 * M2);
    TB_HIP(hipMemcpy(h.data(), c.h, M2 * 8, hipMemcpyDeviceToHost));
    TB_HIP(hipMemcpy(eri.data(), c.eri, M2 * M2 * 8, hipMemcpyDeviceToHost));

    // entries (K, pair, string, sign, slot): string x = K + {a < b}, the
    // slot t numbers x's occupied pairs; sign = (-1)^(n_<a + n_<b - 1)
    const int npo = n * (n - 1) / 2;
    struct E {
        uint64_t K;
        uint32_t pid;
        int32_t x;
        uint32_t neg;
        int32_t t;
    };
    std::vector<E> ent((size_t)l * npo);
    int occ[64];
    for (int64_t x = 0; x < l; ++x) {
        int k = 0;
        for (uint64_t m = str[(size_t)x]; m; m &= m - 1) occ[k++] = __builtin_ctzll(m);
        int t = 0;
        for (int j = 1; j < n; ++j)
            for (int i = 0; i < j; ++i, ++t) {
                const int a = occ[i], b = occ[j];
                const uint64_t K = str[(size_t)x] & ~(1ull << a) & ~(1ull << b);
                ent[(size_t)x * npo + t] = E{K, (uint32_t)pair_id(a, b), (int32_t)x,
                                             (uint32_t)((i + j - 1) & 1), t};
            }
    }
    std::sort(ent.begin(), ent.end(), [](const E &u, const E &v) {
        return u.K != v.K ? u.K < v.K : u.pid < v.pid;
    });
    std::vector<int64_t> ptr;
    std::vector<uint2> he(ent.size());
    std::vector<uint32_t> inv(ent.size());
    int hmax = 0;
    for (size_t e = 0; e < ent.size(); ++e) {
        if (e == 0 || ent[e].K != ent[e - 1].K) {
            if (!ptr.empty()) hmax = std::max(hmax, (int)((int64_t)e - ptr.back()));
            ptr.push_back((int64_t)e);
        }
        he[e] = uint2{(uint32_t)ent[e].x, ent[e].pid | (ent[e].neg << 16)};
        inv[(size_t)ent[e].x * npo + ent[e].t] = (uint32_t)e | (ent[e].neg << 31);
    }
    hmax = std::max(hmax, (int)((int64_t)ent.size() - ptr.back()));
    ptr.push_back((int64_t)ent.size());
    if (hmax > kHoleMax || ent.size() >= (size_t(1) << 31)) return;  // keeps the CSR sweep
    const bool dense = ent.size() >= (size_t)TBSCI_HOLE_AUTO_MIN * (ptr.size() - 1);
    s.hole_auto = dense && large;
    if (!force && !s.hole_auto) return;

    // W[pair(p,r)][pair(q,s)], p < r, q < s
    const int pp = M * (M - 1) / 2;
    auto g = [&](int p, int q, int r, int t) { return eri[((size_t)(p * M + q) * M + r) * M + t]; };
    std::vector<double> W((size_t)pp * pp);
    std::vector<float> W32((size_t)pp * pp);
    const double f = 1.0 / (n - 1);
    for (int r = 1; r < M; ++r)
        for (int p = 0; p < r; ++p)
            for (int t = 1; t < M; ++t)
                for (int q = 0; q < t; ++q) {
                    double v = g(p, q, r, t) - g(p, t, r, q);
                    v += f * ((r == t ? h[p * M + q] : 0.0) + (p == q ? h[r * M + t] : 0.0) -
                              (r == q ? h[p * M + t] : 0.0) - (p == t ? h[r * M + q] : 0.0));
                    const size_t k = (size_t)pair_id(p, r) * pp + pair_id(q, t);
                    W[k] = v;
                    W32[k] = (float)v;
                }
    try {
        s.h_ptr = upload(ptr);
        s.h_ent = upload(he);
        s.h_inv = (int32_t *)upload(inv);
        s.hW = upload(W);
        s.hW32 = upload(W32);
    } catch (...) {
        const bool a = s.hole_auto;
        free_hole(s);
        s.hole_built = true;
        s.hole_auto = a;
        throw;
    }
    s.hmax = hmax;
    s.npo = npo;
    s.pp = pp;
    s.n_hole = (int64_t)ptr.size() - 1;
    s.n_hent = (int64_t)ent.size();
    double mf = 0.0;
    for (size_t k = 0; k + 1 < ptr.size(); ++k) {
        const int64_t nk = ptr[k + 1] - ptr[k];
        mf += (double)((nk + 15) / 16 * 16) * (double)((nk + 3) / 4 * 4);
    }
    s.hole_mfma = mf;
    s.hole = true;
}

// whether a spin's same-spin term takes the hole-pair sweep: always with
// TBSCI_SAME_SPIN_HOLE (when the index exists); with the automatic method
// for the spins hole_build marks, unless a point-group symmetry is set (the
// CSR rows then skip the symmetry-forbidden elements, which the dense pair
// blocks would multiply)
bool hole_on(const Ctx &c, int spin) {
    const Spin &s = c.sp[spin];
    if (!s.hole || c.same_spin == TBSCI_SAME_SPIN_CSR) return false;
    if (c.same_spin == TBSCI_SAME_SPIN_HOLE) return true;
    return s.hole_auto && c.irreps.empty();
}

bool hole_any(const Ctx &c) { return hole_on(c, 0) || hole_on(c, 1); }

// product buffer: the entries of the spins that take the hole-pair sweep
// times the widest window their sweeps use (alpha: l_beta columns; beta:
// the rows of a beta-sweep block), capped at 4 GiB
void *hole_workspace(Ctx &c) {
    size_t need = 0;
    const int64_t la = c.sp[0].l, lb = c.sp[1].l;
    const int64_t ncol[2] = {lb, beta_block_rows(la, lb, kWorkCap)};
    for (int s = 0; s < 2; ++s)
        if (hole_on(c, s))
            need = std::max(need, (size_t)c.sp[s].n_hent * (size_t)((ncol[s] + 63) / 64 * 64) * 8);
    need = std::min(need, kHoleWorkCap);
    if (c.hole_work_bytes < need) {
        if (c.hole_work) TB_HIP(hipFree(c.hole_work));
        c.hole_work = nullptr;
        c.hole_work_bytes = 0;
        TB_HIP(hipMalloc(&c.hole_work, need));
        c.hole_work_bytes = need;
    }
    return c.hole_work;
}

void hole_sweep(Ctx &c, int spin, int64_t ncols, const void *X, void *Y, int precision,
                void *work, size_t work_bytes, hipStream_t st) {
    const Spin &s = c.sp[spin];
    if (precision == TBSCI_FP64)
        hole_sweep_t<double>(s, ncols, (const double *)X, (double *)Y, work, work_bytes, st);
    else
        hole_sweep_t<float>(s, ncols, (const float *)X, (float *)Y, work, work_bytes, st);
}

}  // namespace tbsci
