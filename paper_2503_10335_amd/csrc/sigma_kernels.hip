// sigma = P H P C over the TPB space, split exactly into three terms
// (C and sigma are [l_alpha][l_beta] row-major):
//
//   sigma = A_a C + C A_b^T + sum_{pq,rs} (pq|rs) E^a_pq C (E^b_rs)^T
//
// A_s is the same-spin Hamiltonian between selected strings of spin s
// (paper Sec. II.C: category [2,0] / [0,2] and the one-spin parts of
// [1,0], [0,1], [0,0]); E^s_pq is the single-excitation operator between
// selected strings including p == q (occupation), so the mixed term carries
// [1,1] and the opposite-spin Coulomb parts of [1,0], [0,1], [0,0].  The
// split is exact because the projector onto the TPB space is the tensor
// product of the alpha and beta projectors and the opposite-spin operator
// is a sum of products of one-spin operators.
//
// Kernels of one sigma build:
//   opposite spin : per output alpha row, gather the rows of C linked by
//                   alpha single excitations, multiply by the folded (pq|rs)
//                   block on MFMA, scatter through the beta single lists
//                   into the output row (LDS atomics when it fits in LDS);
//                   the slab kernel when the integral fragments and the row
//                   fit in LDS together, else the same kernel with the
//                   fragments read from the L2-resident integral block;
//   alpha sweep   : sparse rows of A_a times rows of C, one XCD per column
//                   panel so each XCD's L2 holds its panel of C;
//   beta sweep    : the same kernel on C^T, then a transpose-add.
#include <algorithm>
#include <vector>
#include <type_traits>

#include "tbsci_internal.hpp"

namespace tbsci {
namespace {

constexpr int kBlock = 256;
constexpr int kXcd = 8;  // MI355X: 8 XCDs; workgroups are dealt to XCDs round-robin

template <typename T>
struct Vals;
template <>
struct Vals<double> {
    static const double *a(const Spin &s) { return s.a_val; }
    static const double *b(const Spin &s) { return s.b_val; }
    static const double *V(const Ctx &c) { return c.V64; }
};
template <>
struct Vals<float> {
    static const float *a(const Spin &s) { return s.a_val32; }
    static const float *b(const Spin &s) { return s.b_val32; }
    static const float *V(const Ctx &c) { return c.V32; }
};

// ---------------------------------------------------------------- sweeps

// Y[I][c] (+)= sum_e val[e] * X[col[e]][c].  Block = 4 waves = 4 output rows
// x 64 V columns; the list of a row is wave-uniform, X rows are read
// coalesced.  Column tiles belong to XCDs round-robin (tile t on XCD t % 8)
// and an XCD walks its tiles one after the other, so its working set is one
// panel of X (nrows x 64 V columns).
template <typename T, int V>
struct Vec;
template <typename T>
struct Vec<T, 1> {
    typedef T type;
    static __device__ __forceinline__ T zero() { return T(0); }
};
template <typename T>
struct Vec<T, 2> {
    typedef T type __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ type zero() { return type{T(0), T(0)}; }
};
template <typename T>
struct Vec<T, 4> {
    typedef T type __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ type zero() { return type{T(0), T(0), T(0), T(0)}; }
};

// V = columns per lane, a divisor of ncols (so rows start aligned): 2 when
// ncols is even (one 16-byte load per lane per nonzero in FP64), 4 for FP32
// when ncols is a multiple of 4, else 1; a wave covers 64 V columns of its
// row
template <typename T, bool ACC, int V>
__device__ __forceinline__ void row_sweep_block(int64_t b, int64_t nrows, int64_t ncols,
                                                int64_t ntiles, int64_t nrb, int64_t tiles_per_xcd,
                                                const int64_t *__restrict__ ptr,
                                                const int32_t *__restrict__ col,
                                                const T *__restrict__ val,
                                                const T *__restrict__ X, T *__restrict__ Y,
                                                const int32_t *__restrict__ chk = nullptr,
                                                int nch = 1, int ch = 0) {
    using TV = typename Vec<T, V>::type;
    const int64_t xcd = b % kXcd, local = b / kXcd;
    const int64_t tl = local / nrb, rb = local - tl * nrb;
    const int64_t tile = xcd + kXcd * tl;
    if (tl >= tiles_per_xcd || tile >= ntiles) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t I = rb * 4 + wave;
    if (I >= nrows) return;
    const int64_t c = (tile * 64 + lane) * V;
    const bool ok = c < ncols;  // V divides ncols: c + V - 1 < ncols too
    const int64_t ld = ncols / V;
    const TV *__restrict__ Xc = (const TV *)(X + (ok ? c : 0));
    // the row's entries (of source chunk ch when the rows are chunked)
    int64_t e0 = ptr[I], e1 = ptr[I + 1];
    if (chk) {
        const int32_t *o = chk + I * (nch + 1) + ch;
        e1 = e0 + o[1];
        e0 += o[0];
    }
    TV acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = Vec<T, V>::zero();
    int64_t e = e0;
    for (; e + 8 <= e1; e += 8) {
        int32_t j[8];
        T v[8];
        TV x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            j[u] = col[e + u];
            v[u] = val[e + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = Xc[(int64_t)j[u] * ld];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u & 3] += v[u] * x[u];
    }
    for (; e < e1; ++e) acc[0] += val[e] * Xc[(int64_t)col[e] * ld];
    const TV a = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    if (ok) {
        TV *y = (TV *)(Y + I * ncols + c);
        if (ACC)
            *y += a;
        else
            *y = a;
    }
}

// columns per lane for a sweep of ncols columns
__host__ __device__ inline int sweep_vec(int64_t ncols) { return ncols % 2 == 0 ? 2 : 1; }
// FP32 takes 4 columns per lane (16-byte loads) when the rows allow it
template <typename T>
__host__ __device__ inline int sweep_vec_of(int64_t ncols) {
    return (sizeof(T) == 4 && ncols % 4 == 0) ? 4 : sweep_vec(ncols);
}

template <typename T, bool ACC, int V>
__global__ __launch_bounds__(kBlock) void k_row_sweep(int64_t nrows, int64_t ncols, int64_t ntiles,
                                                      int64_t nrb, int64_t tiles_per_xcd,
                                                      const int64_t *__restrict__ ptr,
                                                      const int32_t *__restrict__ col,
                                                      const T *__restrict__ val,
                                                      const T *__restrict__ X, T *__restrict__ Y,
                                                      const int32_t *__restrict__ chk, int nch,
                                                      int ch) {
    row_sweep_block<T, ACC, V>(blockIdx.x, nrows, ncols, ntiles, nrb, tiles_per_xcd, ptr, col, val,
                               X, Y, chk, nch, ch);
}

// Panel sweep: Y (+)= A_s X for one column tile (64 V columns) and a block
// of kPanelBlockRows output rows.  The tile of X is staged in LDS one panel
// of kPanelRows source rows at a time, and each wave accumulates its 4
// output rows from their entries in that panel (the source-chunked CSR), so
// the gathers read LDS instead of L2.  Tiles are dealt to XCDs round-robin,
// so the blocks of one tile stage the same panels out of their XCD's L2.
constexpr int kPanelBlockRows = 64;
constexpr int kPanelThreads = 1024;
constexpr int kPanelRowsPerWave = kPanelBlockRows / (kPanelThreads / 64);

template <typename T, bool ACC, int V>
__global__ __launch_bounds__(kPanelThreads) void k_panel_sweep(
    int64_t nrows, int64_t ncols, int64_t ntiles, int64_t nrb, int64_t tiles_per_xcd,
    const int64_t *__restrict__ ptr, const int32_t *__restrict__ off, int npc,
    const int32_t *__restrict__ col, const T *__restrict__ val, const T *__restrict__ X,
    T *__restrict__ Y) {
    using TV = typename Vec<T, V>::type;
    constexpr int RW = kPanelRowsPerWave;
    __shared__ TV xs[kPanelRows * 64];
    const int64_t b = blockIdx.x;
    const int64_t xcd = b % kXcd, local = b / kXcd;
    const int64_t tl = local / nrb, rb = local - tl * nrb;
    const int64_t tile = xcd + kXcd * tl;
    if (tl >= tiles_per_xcd || tile >= ntiles) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t ld = ncols / V;  // row length of X and Y in TV units
    const TV *__restrict__ Xt = (const TV *)X + tile * 64;
    const int64_t I0 = rb * kPanelBlockRows + wave * RW;
    int64_t base[RW];
    const int32_t *ro[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const bool v = I0 + r < nrows;
        base[r] = v ? ptr[I0 + r] : 0;
        ro[r] = off + (v ? I0 + r : 0) * (npc + 1);
    }
    TV acc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r] = Vec<T, V>::zero();
    for (int ch = 0; ch < npc; ++ch) {
        const int64_t j0 = (int64_t)ch * kPanelRows;
        // stage source rows j0 .. j0 + kPanelRows - 1 of the tile
#pragma unroll
        for (int k = 0; k < kPanelRows * 64 / kPanelThreads; ++k) {
            const int i = tid + k * kPanelThreads;
            const int64_t jr = j0 + (i >> 6);
            const int ln = i & 63;
            TV x = Vec<T, V>::zero();
            if (jr < nrows && tile * 64 + ln < ld) x = Xt[jr * ld + ln];
            xs[i] = x;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            if (I0 + r >= nrows) break;
            int64_t e = base[r] + ro[r][ch];
            const int64_t e1 = base[r] + ro[r][ch + 1];
            for (; e + 4 <= e1; e += 4) {
                int32_t j[4];
                T v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    j[u] = col[e + u] - (int32_t)j0;
                    v[u] = val[e + u];
                }
                TV x[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) x[u] = xs[j[u] * 64 + lane];
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[r] += v[u] * x[u];
            }
            for (; e < e1; ++e) acc[r] += val[e] * xs[(col[e] - (int32_t)j0) * 64 + lane];
        }
        __syncthreads();
    }
    const int64_t cl = tile * 64 + lane;  // this lane's column in TV units
    if (cl < ld) {
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            if (I0 + r >= nrows) break;
            TV *y = (TV *)Y + (I0 + r) * ld + cl;
            if (ACC)
                *y += acc[r];
            else
                *y = acc[r];
        }
    }
}

// Descriptor of one problem in a grouped launch; the problem's blocks are
// [blk0, blk0 + its block count), blk0 a multiple of 8 so that the XCD of a
// block is the same as in a launch of its own.
struct SweepDesc {
    int64_t blk0, nrows, ncols, ntiles, nrb, tpx;
    const int64_t *ptr;
    const int32_t *col;
    const void *val, *X;
    void *Y;
};

// index of the descriptor whose block range holds block b (blk0 ascending)
template <typename D>
__device__ __forceinline__ int find_desc(const D *__restrict__ d, int nd, int64_t b) {
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].blk0 <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <typename T, bool ACC>
__global__ __launch_bounds__(kBlock) void g_row_sweep(const SweepDesc *__restrict__ d, int nd) {
    const SweepDesc e = d[find_desc(d, nd, blockIdx.x)];
    const int vec = sweep_vec_of<T>(e.ncols);
    if (vec == 4)
        row_sweep_block<T, ACC, 4>(blockIdx.x - e.blk0, e.nrows, e.ncols, e.ntiles, e.nrb, e.tpx,
                                   e.ptr, e.col, (const T *)e.val, (const T *)e.X, (T *)e.Y);
    else if (vec == 2)
        row_sweep_block<T, ACC, 2>(blockIdx.x - e.blk0, e.nrows, e.ncols, e.ntiles, e.nrb, e.tpx,
                                   e.ptr, e.col, (const T *)e.val, (const T *)e.X, (T *)e.Y);
    else
        row_sweep_block<T, ACC, 1>(blockIdx.x - e.blk0, e.nrows, e.ncols, e.ntiles, e.nrb, e.tpx,
                                   e.ptr, e.col, (const T *)e.val, (const T *)e.X, (T *)e.Y);
}

// out[c][r] (+)= in[r][c] for an R x Cn row-major input; 32 x 32 tiles via LDS.
template <typename T, bool ADD>
__device__ __forceinline__ void transpose_block(int64_t b, int64_t R, int64_t Cn, int64_t ntc,
                                                const T *__restrict__ in, T *__restrict__ out) {
    __shared__ T tile[32][33];
    const int64_t tr = b / ntc, tc = b - tr * ntc;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
    for (int i = ty; i < 32; i += 8) {
        const int64_t r = tr * 32 + i, c = tc * 32 + tx;
        if (r < R && c < Cn) tile[i][tx] = in[r * Cn + c];
    }
    __syncthreads();
#pragma unroll
    for (int i = ty; i < 32; i += 8) {
        const int64_t c = tc * 32 + i, r = tr * 32 + tx;
        if (r < R && c < Cn) {
            const T v = tile[tx][i];
            if (ADD)
                out[c * R + r] += v;
            else
                out[c * R + r] = v;
        }
    }
}

template <typename T, bool ADD>
__global__ __launch_bounds__(kBlock) void k_transpose(int64_t R, int64_t Cn, int64_t ntc,
                                                      const T *__restrict__ in, T *__restrict__ out) {
    transpose_block<T, ADD>(blockIdx.x, R, Cn, ntc, in, out);
}

struct TransDesc {
    int64_t blk0, R, Cn, ntc;
    const void *in;
    void *out;
};

template <typename T, bool ADD>
__global__ __launch_bounds__(kBlock) void g_transpose(const TransDesc *__restrict__ d, int nd) {
    const TransDesc e = d[find_desc(d, nd, blockIdx.x)];
    transpose_block<T, ADD>(blockIdx.x - e.blk0, e.R, e.Cn, e.ntc, (const T *)e.in, (T *)e.out);
}

// ---------------------------------------------------------- opposite spin

template <typename T>
struct Mfma;
// Operand layouts of the 16x16x4 MFMAs (lane l, 0..63): A[m][k] with
// m = l%16, k = l/16; B[k][n] with k = l/16, n = l%16.  Accumulator register
// r of lane l holds D[row(l, r)][l%16]; the row order differs by type.
template <>
struct Mfma<double> {
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma<float> {
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// Per output alpha row I and beta string c:
//
//   X[k][c]  = C[J_k][c]                     (gathered, k over the alpha links
//                                              of I)
//   Y[rs][c] = sum_k s_k V[pq_k][rs] X[k][c]  (MFMA over 16-pair M-tiles)
//   row[I']  += s * Y[pair][J']  for every link (I', pair, s) of J' in the
//               beta single lists (symmetric: the links of J' are the
//               sources of I')
//
// Y never leaves the accumulators: the A rows are ordered so that register r
// of a lane in lane group g holds pair 16 m + 4 r + g of its column, and the
// links are grouped by (tile, g), so each lane reads just its own links.
//
// ROW selects where the output row accumulates: an FP64 row in LDS (FP64
// LDS atomics, also for FP32 sigma: on gfx950 they are several times faster
// than FP32 LDS atomics, and the row is rounded once at the end) for as many
// beta strings as fit, the rest through global atomics on sigma; or, for an
// FP32 row too long for that, a whole row of type T in LDS.
template <typename T>
__device__ __forceinline__ int a_row_pair(int m);  // pair (within the tile) of A row m
template <>
__device__ __forceinline__ int a_row_pair<double>(int m) {
    return m;  // FP64 accumulator: row m = 4 r + g
}
template <>
__device__ __forceinline__ int a_row_pair<float>(int m) {
    return 4 * (m & 3) + (m >> 2);  // FP32 accumulator: row m = 4 g + r
}

template <typename V4>
__device__ __forceinline__ auto pick4(const V4 &v, int r) {
    return r == 0 ? v[0] : r == 1 ? v[1] : r == 2 ? v[2] : v[3];
}

// Where the output row accumulates: kRowF64, a whole FP64 row in LDS;
// kRowSplit, an FP64 row in LDS for the first nrow beta strings, the links
// to strings beyond nrow going to sigma through global atomics; kRowSplitT,
// the same with a row of type T (an FP32 sigma keeps twice as many entries
// in LDS); kRowT, a
// whole row of type T in LDS
enum { kRowF64 = 0, kRowT = 1, kRowSplit = 2, kRowSplitT = 3 };

constexpr size_t kLdsMax = 160 * 1024;

// Slab kernel: one output row I per block, waves independent of each other.
// The A fragments of every M-tile (the signed integral rows U of the alpha
// links of I) are staged in LDS once per row.  A wave takes 16-column slabs
// of beta strings off a counter in LDS; per slab it loads its B fragments
// (C[J_k][16 columns]) straight from global
// memory into registers and runs the M-tiles one after another: MFMA over
// the links, then the scatter of the tile's accumulators through the beta
// single lists into the FP64 row in LDS.  There is no barrier between
// slabs, so one wave's MFMAs overlap other waves' loads and LDS atomics;
// each C element is loaded once per row, by the wave that owns its slab.
// LDS holds the whole FP64 row plus ceil(P/16) x ceil(K_max/4) fragments.
struct SlabLds {
    size_t row, a, aj, ctr, total;
};

inline SlabLds slab_lds(int64_t lb, int nmt, int nks, size_t sz) {
    SlabLds L{};
    size_t o = 0;
    auto take = [&](size_t n) {
        const size_t at = o;
        o += (n + 15) & ~size_t(15);
        return at;
    };
    const int nk4 = (nks + 3) / 4 * 4;  // k-steps padded to the largest chunk
    L.row = take((size_t)lb * 8);
    L.a = take((size_t)nmt * nk4 * 64 * sz);
    L.aj = take((size_t)nk4 * 4 * 4);
    L.ctr = take(4);
    L.total = o;
    return L;
}

// Deterministic accumulation of the output row: with det != null the row
// holds 64-bit fixed-point values, each contribution v added as
// round(v * scale) with integer atomics (associative, so the sum does not
// depend on the order of the adds); scale = *det, a power of two chosen so
// that no partial sum can leave the 63-bit range (k_det_scale).
__device__ __forceinline__ unsigned long long to_fixed(double v, double scale) {
    return (unsigned long long)__double2ll_rn(v * scale);
}
__device__ __forceinline__ double from_fixed(unsigned long long a, double scale) {
    return (double)(long long)a / scale;
}

template <typename T, int KS>
__device__ __forceinline__ void ab_slab_row(const int64_t I, int64_t lb, int P, int nmt,
                                            const SlabLds L, const int64_t *__restrict__ sa_ptr,
                                            const Ent *__restrict__ sa_ent,
                                            const int64_t *__restrict__ sb_ptr,
                                            const Ent *__restrict__ sb_grp,
                                            const int32_t *__restrict__ sb_off,
                                            const T *__restrict__ V, const T *__restrict__ C,
                                            T *__restrict__ S, const double *__restrict__ det) {
    using M = Mfma<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    double *row = (double *)(smem + L.row);
    unsigned long long *rowi = (unsigned long long *)(smem + L.row);
    const double dscale = det ? *det : 0.0;
    T *afr = (T *)(smem + L.a);
    int32_t *aj = (int32_t *)(smem + L.aj);
    int *ctr = (int *)(smem + L.ctr);

    const int nthr = blockDim.x, tid = threadIdx.x, lane = tid & 63;
    const int g = lane >> 4, cl = lane & 15;
    const int64_t a0 = sa_ptr[I];
    const int K = (int)(sa_ptr[I + 1] - a0);
    // k-steps of 4 links, run in chunks of CK MFMAs (padding steps hold
    // zero fragments); FP32 takes chunks of 4 with the C loads of a chunk
    // issued together, FP64 single steps (its MFMA time dominates, padding
    // would add to it)
    constexpr int CK = sizeof(T) == 8 ? 1 : 4;
    const int nks = (((K + 3) >> 2) + CK - 1) / CK * CK;
    const int ng = 4 * nmt;

    for (int64_t i = tid; i < lb; i += nthr) row[i] = 0.0;
    for (int k = tid; k < 4 * nks; k += nthr) aj[k] = k < K ? sa_ent[a0 + k].j : -1;
    // A fragment (m, ks), lane ln: U[k = 4 ks + ln/16][pair of row ln%16 of tile m]
    const int na = nmt * nks * 64;
    for (int i = tid; i < na; i += nthr) {
        const int ln = i & 63, q = i >> 6;
        const int m = q / nks, ks = q - m * nks;
        const int k = 4 * ks + (ln >> 4);
        const int pr = 16 * m + a_row_pair<T>(ln & 15);
        T a = T(0);
        if (k < K && pr < P) {
            const Ent e = sa_ent[a0 + k];
            const T v = V[(int64_t)(e.o >> 16) * P + pr];
            a = ((e.o >> 12) & 1u) ? -v : v;
        }
        afr[i] = a;
    }
    if (tid == 0) *ctr = 0;
    __syncthreads();

    const int64_t nslab = (lb + 15) >> 4;
    for (;;) {
        int sl = 0;
        if (lane == 0) sl = atomicAdd(ctr, 1);
        sl = __builtin_amdgcn_readfirstlane(sl);
        if (sl >= nslab) break;
        const int64_t col = (int64_t)sl * 16 + cl;
        const bool cin = col < lb;
        T b[KS];
        if constexpr (CK == 1) {
            // the link rows first (one LDS round trip), then the loads
            int32_t J[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) J[ks] = ks < nks ? aj[4 * ks + g] : -1;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                T v = T(0);
                if (J[ks] >= 0 && cin) v = C[(int64_t)J[ks] * lb + col];
                b[ks] = v;
            }
        } else {
#pragma unroll
            for (int q = 0; q < KS / CK; ++q)
                if (CK * q < nks) {
                    int32_t J[CK];
#pragma unroll
                    for (int u = 0; u < CK; ++u) J[u] = aj[4 * (CK * q + u) + g];
#pragma unroll
                    for (int u = 0; u < CK; ++u) {  // in-bounds load, then select
                        const bool ok = J[u] >= 0 && cin;
                        const T v = C[ok ? (int64_t)J[u] * lb + col : 0];
                        b[CK * q + u] = ok ? v : T(0);
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < CK; ++u) b[CK * q + u] = T(0);
                }
        }
        const int32_t *off = sb_off + (cin ? col : 0) * (ng + 1) + g;
        const int64_t base = cin ? sb_ptr[col] : 0;
        int32_t n0 = 0, n1 = 0;  // link range of the next tile
        if (cin) {
            n0 = off[0];
            n1 = off[1];
        }
        for (int m = 0; m < nmt; ++m) {
            const int32_t o0 = n0, o1 = n1;
            // the first four links of this tile and the next tile's range are
            // loaded before the MFMAs, so they arrive while those run
            Ent e0{0, 0}, e1{0, 0}, e2{0, 0}, e3{0, 0};
            const bool h0 = o0 < o1, h1 = o0 + 1 < o1, h2 = o0 + 2 < o1, h3 = o0 + 3 < o1;
            if (h0) e0 = sb_grp[base + o0];
            if (h1) e1 = sb_grp[base + o0 + 1];
            if (h2) e2 = sb_grp[base + o0 + 2];
            if (h3) e3 = sb_grp[base + o0 + 3];
            if (cin && m + 1 < nmt) {
                n0 = off[4 * (m + 1)];
                n1 = off[4 * (m + 1) + 1];
            }
            typename M::acc_t acc = typename M::acc_t{0, 0, 0, 0};
            const T *am = afr + (size_t)m * nks * 64 + lane;
#pragma unroll
            for (int q = 0; q < KS / CK; ++q)
                if (CK * q < nks) {
                    T a[CK];
#pragma unroll
                    for (int u = 0; u < CK; ++u) a[u] = am[(CK * q + u) * 64];
#pragma unroll
                    for (int u = 0; u < CK; ++u) acc = M::mma(a[u], b[CK * q + u], acc);
                }
            // register r holds pair 16 m + 4 r + g of this lane's column
            auto put = [&](const Ent &e) {
                T v = pick4(acc, (int)(((e.o >> 16) & 15) >> 2));
                if ((e.o >> 12) & 1u) v = -v;
                if (det)
                    atomicAdd(&rowi[e.j], to_fixed((double)v, dscale));
                else
                    atomicAdd(&row[e.j], (double)v);
            };
            if (h0) put(e0);
            if (h1) put(e1);
            if (h2) put(e2);
            if (h3) put(e3);
            for (int32_t x = o0 + 4; x < o1; ++x) put(sb_grp[base + x]);
        }
    }
    __syncthreads();
    if (det)
        for (int64_t i = tid; i < lb; i += nthr)
            S[I * lb + i] = (T)((double)S[I * lb + i] + from_fixed(rowi[i], dscale));
    else
        for (int64_t i = tid; i < lb; i += nthr)
            S[I * lb + i] = (T)((double)S[I * lb + i] + row[i]);
}

constexpr int kSlabBlock = 1024;

template <typename T, int KS>
__global__ __launch_bounds__(kSlabBlock) void k_ab_slab(int64_t lb, int P, int nmt, SlabLds L,
                                                       const int64_t *__restrict__ sa_ptr,
                                                       const Ent *__restrict__ sa_ent,
                                                       const int64_t *__restrict__ sb_ptr,
                                                       const Ent *__restrict__ sb_grp,
                                                       const int32_t *__restrict__ sb_off,
                                                       const T *__restrict__ V,
                                                       const T *__restrict__ C,
                                                       T *__restrict__ S,
                                                       const double *__restrict__ det) {
    ab_slab_row<T, KS>(blockIdx.x, lb, P, nmt, L, sa_ptr, sa_ent, sb_ptr, sb_grp, sb_off, V, C,
                       S, det);
}

// Slab kernel with the A fragments read from global memory, for rows whose
// fragments do not fit LDS beside the output row.  The sign of each alpha
// link is folded into its C fragment, so an A fragment is a plain element
// of the folded integral block V (L2-resident): lane l of k-step ks reads
// V[pq_k][16 m + row(l)] with k = 4 ks + l/16.  LDS holds the output row
// (whole, split, or of type T: see ROW above) and the link columns.
struct SlabgLds {
    size_t row, aj, apq, ctr, total;
    int64_t nrow;  // row entries held in LDS
};

inline SlabgLds slabg_lds(int64_t lb, int nks, size_t row_sz, int64_t nrow = -1) {
    SlabgLds L{};
    size_t o = 0;
    auto take = [&](size_t n) {
        const size_t at = o;
        o += (n + 15) & ~size_t(15);
        return at;
    };
    const int nk4 = (nks + 3) / 4 * 4;
    L.aj = take((size_t)nk4 * 4 * 4);
    L.apq = take((size_t)nk4 * 4 * 4);
    L.ctr = take(4);
    if (nrow < 0) {
        const size_t room = o < kLdsMax ? (kLdsMax - o) / row_sz : 0;
        nrow = std::min<int64_t>(lb, (int64_t)(room & ~size_t(1)));
    }
    L.nrow = nrow;
    L.row = take((size_t)nrow * row_sz);
    L.total = o;
    return L;
}

template <typename T, int KS, int ROW>
__device__ __forceinline__ void ab_slabg_row(const int64_t I, int64_t lb, int P, int nmt,
                                             const SlabgLds L, const int64_t *__restrict__ sa_ptr,
                                             const Ent *__restrict__ sa_ent,
                                             const int64_t *__restrict__ sb_ptr,
                                             const Ent *__restrict__ sb_grp,
                                             const int32_t *__restrict__ sb_off,
                                             const T *__restrict__ V, const T *__restrict__ C,
                                             T *__restrict__ S, const double *__restrict__ det,
                                             unsigned long long *__restrict__ stage) {
    using M = Mfma<T>;
    using R = typename std::conditional<ROW == kRowT || ROW == kRowSplitT, T, double>::type;
    constexpr bool kSplit = ROW == kRowSplit || ROW == kRowSplitT;
    const int64_t nrow = kSplit ? L.nrow : lb;
    extern __shared__ __align__(16) unsigned char smem[];
    R *row = (R *)(smem + L.row);
    // fixed-point row (det): the 8-byte row in LDS, and for a split row the
    // rest in this row's segment of the fixed-point staging area
    unsigned long long *rowi = (unsigned long long *)(smem + L.row);
    const bool fixed = (ROW == kRowF64 || ROW == kRowSplit) && det;
    const double dscale = fixed ? *det : 0.0;
    unsigned long long *srow = fixed && kSplit ? stage + I * (lb - nrow) : nullptr;
    int32_t *aj = (int32_t *)(smem + L.aj);
    int32_t *apq = (int32_t *)(smem + L.apq);
    int *ctr = (int *)(smem + L.ctr);

    const int nthr = blockDim.x, tid = threadIdx.x, lane = tid & 63;
    const int g = lane >> 4, cl = lane & 15;
    const int64_t a0 = sa_ptr[I];
    const int K = (int)(sa_ptr[I + 1] - a0);
    const int nks = (K + 3) >> 2;
    const int ng = 4 * nmt;
    constexpr int G = 4;  // A fragments loaded per group, one group ahead

    // link columns, laid out [lane group][k-step] so that a lane's four
    // consecutive k-steps are one 16-byte LDS read: aj = source row J (or
    // -1), apq = pq_k P (the V row offset) | sign << 30
    const int nk4 = (nks + 3) & ~3;
    for (int64_t i = tid; i < nrow; i += nthr) row[i] = R(0);
    for (int k = tid; k < 4 * nk4; k += nthr) {
        int32_t J = -1, pq = 0;
        if (k < K) {
            const Ent e = sa_ent[a0 + k];
            J = e.j;
            pq = (int32_t)((e.o >> 16) * (uint32_t)P) | (int32_t)(((e.o >> 12) & 1u) << 30);
        }
        const int kk = (k & 3) * nk4 + (k >> 2);  // k = 4 ks + g -> [g][ks]
        aj[kk] = J;
        apq[kk] = pq;
    }
    if (tid == 0) *ctr = 0;
    __syncthreads();

    const int32_t *ajg = aj + g * nk4, *apg = apq + g * nk4;
    uint32_t sgn = 0;  // link signs of this lane's k-steps
    for (int ks = 0; ks < nks; ++ks) sgn |= (uint32_t)((apg[ks] >> 30) & 1) << ks;

    const int r16 = a_row_pair<T>(cl);
    const int64_t nslab = (lb + 15) >> 4;
    for (;;) {
        int sl = 0;
        if (lane == 0) sl = atomicAdd(ctr, 1);
        sl = __builtin_amdgcn_readfirstlane(sl);
        if (sl >= nslab) break;
        const int64_t col = (int64_t)sl * 16 + cl;
        const bool cin = col < lb;
        // C fragments of all KS k-steps, without branches: every load goes to
        // a valid address (element 0 for steps past the list or columns past
        // lb) and is replaced by zero when used, so no wait is forced early
        T b[KS];
        {
            int32_t J[KS];
#pragma unroll
            for (int q = 0; q < KS / 4; ++q) {
                const int4 j4 = *(const int4 *)(ajg + std::min(4 * q, std::max(nk4 - 4, 0)));
                const int jj[4] = {j4.x, j4.y, j4.z, j4.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) J[4 * q + u] = 4 * q + u < nk4 ? jj[u] : -1;
            }
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                b[ks] = C[(J[ks] >= 0 && cin) ? (int64_t)J[ks] * lb + col : 0];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const T x = (J[ks] >= 0 && cin) ? b[ks] : T(0);
                b[ks] = ((sgn >> ks) & 1u) ? -x : x;
            }
        }
        const int32_t *off = sb_off + (cin ? col : 0) * (ng + 1) + g;
        const int64_t base = cin ? sb_ptr[col] : 0;
        int32_t n0 = 0, n1 = 0;
        if (cin) {
            n0 = off[0];
            n1 = off[1];
        }
        for (int m = 0; m < nmt; ++m) {
            const int32_t o0 = n0, o1 = n1;
            Ent e0{0, 0}, e1{0, 0}, e2{0, 0}, e3{0, 0};
            const bool h0 = o0 < o1, h1 = o0 + 1 < o1, h2 = o0 + 2 < o1, h3 = o0 + 3 < o1;
            if (h0) e0 = sb_grp[base + o0];
            if (h1) e1 = sb_grp[base + o0 + 1];
            if (h2) e2 = sb_grp[base + o0 + 2];
            if (h3) e3 = sb_grp[base + o0 + 3];
            if (cin && m + 1 < nmt) {
                n0 = off[4 * (m + 1)];
                n1 = off[4 * (m + 1) + 1];
            }
            // this lane's column of V for tile m (row 0 stands in for pairs
            // past P: those accumulator rows are never scattered)
            const int pr = 16 * m + r16;
            const T *Vm = V + (pr < P ? pr : 0);
            // A fragments of k-step group q: V[pq_k P + pr] for the group's
            // four k-steps; steps past the list read offset 0 (their C
            // fragments are zero).  All KS steps run, without branches.
            auto ldg = [&](int q, T *a) {
                int4 o4 = *(const int4 *)(apg + std::min(4 * q, std::max(nk4 - 4, 0)));
                if (4 * q >= nk4) o4 = make_int4(0, 0, 0, 0);
                a[0] = Vm[o4.x & 0xffff];
                a[1] = Vm[o4.y & 0xffff];
                a[2] = Vm[o4.z & 0xffff];
                a[3] = Vm[o4.w & 0xffff];
            };
            typename M::acc_t acc = typename M::acc_t{0, 0, 0, 0};
            T an[G];
            ldg(0, an);
#pragma unroll
            for (int q = 0; q < KS / G; ++q) {
                T a[G];
#pragma unroll
                for (int u = 0; u < G; ++u) a[u] = an[u];
                if (q + 1 < KS / G) ldg(q + 1, an);
#pragma unroll
                for (int u = 0; u < G; ++u) acc = M::mma(a[u], b[G * q + u], acc);
            }
            auto put = [&](const Ent &e) {
                T v = pick4(acc, (int)(((e.o >> 16) & 15) >> 2));
                if ((e.o >> 12) & 1u) v = -v;
                if (fixed)
                    atomicAdd(!kSplit || e.j < nrow ? &rowi[e.j] : &srow[e.j - nrow],
                              to_fixed((double)v, dscale));
                else if (!kSplit || e.j < nrow)
                    atomicAdd(&row[e.j], (R)v);
                else
                    atomicAdd(&S[I * lb + e.j], v);
            };
            if (h0) put(e0);
            if (h1) put(e1);
            if (h2) put(e2);
            if (h3) put(e3);
            for (int32_t x = o0 + 4; x < o1; ++x) put(sb_grp[base + x]);
        }
    }
    // the staged part of a split row: every add to it came from this block;
    // the fence makes them complete at device scope before they are read
    // back (and the segment cleared for the next call) with exchanges
    if (fixed && kSplit) __threadfence();
    __syncthreads();
    if (fixed) {
        for (int64_t i = tid; i < nrow; i += nthr)
            S[I * lb + i] = (T)((double)S[I * lb + i] + from_fixed(rowi[i], dscale));
        if (kSplit)
            for (int64_t i = nrow + tid; i < lb; i += nthr)
                S[I * lb + i] =
                    (T)((double)S[I * lb + i] +
                        from_fixed(atomicExch(&srow[i - nrow], 0ull), dscale));
    } else
        for (int64_t i = tid; i < nrow; i += nthr)
            S[I * lb + i] = (T)((R)S[I * lb + i] + row[i]);
}

template <typename T, int KS, int ROW>
__global__ __launch_bounds__(kSlabBlock) void k_ab_slabg(int64_t lb, int P, int nmt, SlabgLds L,
                                                        const int64_t *__restrict__ sa_ptr,
                                                        const Ent *__restrict__ sa_ent,
                                                        const int64_t *__restrict__ sb_ptr,
                                                        const Ent *__restrict__ sb_grp,
                                                        const int32_t *__restrict__ sb_off,
                                                        const T *__restrict__ V,
                                                        const T *__restrict__ C,
                                                        T *__restrict__ S,
                                                        const double *__restrict__ det,
                                                        unsigned long long *__restrict__ stage,
                                                        const int32_t *__restrict__ rows) {
    ab_slabg_row<T, KS, ROW>(rows[blockIdx.x], lb, P, nmt, L, sa_ptr, sa_ent, sb_ptr, sb_grp,
                             sb_off, V, C, S, det, stage);
}

// one problem of a grouped slab launch: blocks [blk0, blk0 + l_alpha)
struct SlabDesc {
    int64_t blk0, lb;
    SlabLds L;
    const int64_t *sa_ptr;
    const Ent *sa_ent;
    const int64_t *sb_ptr;
    const Ent *sb_grp;
    const int32_t *sb_off;
    const void *V, *C;
    void *S;
    const double *det;  // fixed-point scale of the problem (deterministic mode) or null
};

template <typename T, int KS>
__global__ __launch_bounds__(kSlabBlock) void g_ab_slab(const SlabDesc *__restrict__ d, int nd,
                                                       int P, int nmt) {
    const SlabDesc e = d[find_desc(d, nd, blockIdx.x)];
    ab_slab_row<T, KS>(blockIdx.x - e.blk0, e.lb, P, nmt, e.L, e.sa_ptr, e.sa_ent, e.sb_ptr,
                       e.sb_grp, e.sb_off, (const T *)e.V, (const T *)e.C, (T *)e.S, e.det);
}

// ---------------------------------------------------------------- driver

// the context's beta-sweep workspace (sigma_work_bytes), allocated on
// first use
// whether a problem may share the grouped launches of a batch: its beta
// sweep in one block, and the CSR sweeps for both spins
bool groupable(const Ctx &c) {
    return !hole_any(c) && beta_block_rows(c.sp[0].l, c.sp[1].l, kWorkCap) >= c.sp[0].l;
}

void *ctx_workspace(Ctx &c) {
    const size_t need = sigma_work_bytes(c.sp[0].l, c.sp[1].l);
    if (c.work_bytes < need) {
        if (c.work) TB_HIP(hipFree(c.work));
        c.work = nullptr;
        c.work_bytes = 0;
        TB_HIP(hipMalloc(&c.work, need));
        c.work_bytes = need;
    }
    return c.work;
}

// o[i] = 0 for i < n (a kernel rather than a memset node, so that the
// sigma launches can be captured into a graph)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_zero(int64_t n, T *__restrict__ o) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        o[i] = T(0);
}

template <typename T>
void launch_zero(int64_t n, T *o, hipStream_t st) {
    if (n <= 0) return;
    const int64_t g = std::min<int64_t>((n + kBlock - 1) / kBlock, 8192);
    k_zero<T><<<(unsigned)g, kBlock, 0, st>>>(n, o);
    TB_HIP(hipGetLastError());
}

// Y (+)= A_s X.  With more than one source chunk, one pass per chunk (the
// first one writes unless acc), so that the X rows an XCD gathers in a pass
// stay in its L2.
template <typename T>
void launch_row_sweep(const Spin &s, int64_t ncols, const T *X, T *Y, bool acc, hipStream_t st,
                      bool fixed_order = false) {
    const int64_t nrows = s.l;
    const int vec = sweep_vec_of<T>(ncols);
    // one launch, panels staged in LDS: FP64, and FP32 with 4 columns per
    // lane (16-byte row segments like FP64; with 2 columns per lane FP32
    // measured faster with the plain sweep out of L2).  fixed_order: one
    // plain pass over the whole rows, the summation order of the grouped
    // sweep (deterministic sigma, equal alone and in a batch)
    if (!fixed_order && s.chunk == kPanelRows && (sizeof(T) == 8 || vec == 4)) {
        const int64_t ntiles = (ncols + 64 * vec - 1) / (64 * vec);
        const int64_t nrb = (nrows + kPanelBlockRows - 1) / kPanelBlockRows;
        const int64_t tpx = (ntiles + kXcd - 1) / kXcd;
        const unsigned grid = (unsigned)(kXcd * tpx * nrb);
        auto f = vec == 4   ? (acc ? k_panel_sweep<T, true, 4> : k_panel_sweep<T, false, 4>)
                 : vec == 2 ? (acc ? k_panel_sweep<T, true, 2> : k_panel_sweep<T, false, 2>)
                            : (acc ? k_panel_sweep<T, true, 1> : k_panel_sweep<T, false, 1>);
        f<<<grid, kPanelThreads, 0, st>>>(nrows, ncols, ntiles, nrb, tpx, s.a_ptr, s.b_off,
                                          s.nch, s.b_col, Vals<T>::b(s), X, Y);
        TB_HIP(hipGetLastError());
        return;
    }
    const int64_t ntiles = (ncols + 64 * vec - 1) / (64 * vec), nrb = (nrows + 3) / 4;
    const int64_t tpx = (ntiles + kXcd - 1) / kXcd;
    const unsigned grid = (unsigned)(kXcd * tpx * nrb);
    const bool chunked = !fixed_order && s.chunk == kSweepChunk && s.nch > 1;
    const int nch = chunked ? s.nch : 1;
    for (int ch = 0; ch < nch; ++ch) {
        const bool a = acc || ch > 0;
        auto f = vec == 4   ? (a ? k_row_sweep<T, true, 4> : k_row_sweep<T, false, 4>)
                 : vec == 2 ? (a ? k_row_sweep<T, true, 2> : k_row_sweep<T, false, 2>)
                            : (a ? k_row_sweep<T, true, 1> : k_row_sweep<T, false, 1>);
        f<<<grid, kBlock, 0, st>>>(nrows, ncols, ntiles, nrb, tpx, s.a_ptr,
                                   chunked ? s.b_col : s.a_col,
                                   chunked ? Vals<T>::b(s) : Vals<T>::a(s), X, Y,
                                   chunked ? s.b_off : nullptr, s.nch, ch);
        TB_HIP(hipGetLastError());
    }
}

template <typename T, bool ADD>
void launch_transpose(int64_t R, int64_t Cn, const T *in, T *out, hipStream_t st) {
    const int64_t ntr = (R + 31) / 32, ntc = (Cn + 31) / 32;
    k_transpose<T, ADD><<<(unsigned)(ntr * ntc), kBlock, 0, st>>>(R, Cn, ntc, in, out);
    TB_HIP(hipGetLastError());
}

// raise a kernel's dynamic LDS limit once per context and kernel
void allow_lds(Ctx &c, const void *f, size_t bytes) {
    for (auto &e : c.lds_set)
        if (e.first == f && e.second >= bytes) return;
    TB_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    c.lds_set.emplace_back(f, bytes);
}

// whether the global-fragment slab kernel takes a context: k-steps within
// its register budget, and V row offsets pq P that fit 16 bits
bool slabg_fits(const Ctx &c) {
    const int ks = std::max((c.sp[0].max_s + 3) / 4, 1);
    return ks <= 32 && c.P * c.P < 65536;
}

template <typename T, int KS>
void launch_ab_slabg_class(Ctx &c, int row, const SlabgLds &L, const int32_t *rows,
                           int64_t n, const T *C, T *S, hipStream_t st) {
    const Spin &A = c.sp[0], &B = c.sp[1];
    const int P = c.P, nmt = (P + 15) / 16;
    auto f = row == kRowF64      ? k_ab_slabg<T, KS, kRowF64>
             : row == kRowT      ? k_ab_slabg<T, KS, kRowT>
             : row == kRowSplitT ? k_ab_slabg<T, KS, kRowSplitT>
                                 : k_ab_slabg<T, KS, kRowSplit>;
    if (L.total > 64 * 1024) allow_lds(c, (const void *)f, L.total);
    f<<<(unsigned)n, kSlabBlock, L.total, st>>>(B.l, P, nmt, L, A.s_ptr, A.s_ent, B.s_ptr,
                                                B.g_ent, B.g_off, Vals<T>::V(c), C, S,
                                                c.det ? c.det_buf + 1 : nullptr,
                                                c.det ? c.det_stage : nullptr, rows);
    TB_HIP(hipGetLastError());
}

// The global-fragment kernel runs a fixed number of k-steps per row (no
// branches in its MFMA loop), so the alpha rows go in classes by their own
// k-step count (8, 16, 24, 28, 32; lists built at create time), one launch
// per class, all with the LDS layout of the longest list.
template <typename T>
void launch_ab_slabg(Ctx &c, const T *C, T *S, hipStream_t st) {
    const Spin &A = c.sp[0], &B = c.sp[1];
    const int ks = std::max((A.max_s + 3) / 4, 1);
    // an FP64 row (split when the whole row does not fit); FP32 sigma with
    // a long row keeps a whole FP32 row instead when that fits
    int row = kRowF64;
    SlabgLds L = slabg_lds(B.l, ks, 8);
    if (L.nrow < B.l) {
        row = kRowSplit;
        // deterministic mode keeps the 8-byte fixed-point row in every precision
        if (sizeof(T) < 8 && !c.det) {
            // an FP32 sigma keeps a whole FP32 row when that fits, else the
            // longer FP32 part of a split row
            const SlabgLds Lt = slabg_lds(B.l, ks, sizeof(T), B.l);
            if (Lt.total <= kLdsMax) {
                row = kRowT;
                L = Lt;
            } else {
                row = kRowSplitT;
                L = slabg_lds(B.l, ks, sizeof(T));
            }
        }
    }
    if (c.det && row == kRowSplit &&
        (!c.det_stage || c.det_stage_n < A.l * (B.l - L.nrow)))
        throw Error(TBSCI_E_STATE, "deterministic sigma: the fixed-point staging area is missing");
    if (!A.ks_rows) throw Error(TBSCI_E_STATE, "alpha row classes missing");
    const int64_t *o = A.ks_off;
    const int32_t *r = A.ks_rows;
    if (o[1] > o[0]) launch_ab_slabg_class<T, 8>(c, row, L, r + o[0], o[1] - o[0], C, S, st);
    if (o[2] > o[1]) launch_ab_slabg_class<T, 16>(c, row, L, r + o[1], o[2] - o[1], C, S, st);
    if (o[3] > o[2]) launch_ab_slabg_class<T, 24>(c, row, L, r + o[2], o[3] - o[2], C, S, st);
    if (o[4] > o[3]) launch_ab_slabg_class<T, 28>(c, row, L, r + o[3], o[4] - o[3], C, S, st);
    if (o[5] > o[4]) launch_ab_slabg_class<T, 32>(c, row, L, r + o[4], o[5] - o[4], C, S, st);
}

// KS instance of the slab kernel for a context (0: it does not apply)
int slab_ks(const Ctx &c, size_t sz) {
    const int ks = std::max((c.sp[0].max_s + 3) / 4, 1);
    if (ks > 24) return 0;
    if (slab_lds(c.sp[1].l, (c.P + 15) / 16, ks, sz).total > kLdsMax) return 0;
    return (ks + 3) / 4 * 4;
}

template <typename T, int KS>
void launch_ab_slab(Ctx &c, const T *C, T *S, hipStream_t st) {
    const Spin &A = c.sp[0], &B = c.sp[1];
    const int P = c.P, nmt = (P + 15) / 16;
    const SlabLds L = slab_lds(B.l, nmt, std::max((A.max_s + 3) / 4, 1), sizeof(T));
    auto f = k_ab_slab<T, KS>;
    if (L.total > 64 * 1024) allow_lds(c, (const void *)f, L.total);
    f<<<(unsigned)A.l, kSlabBlock, L.total, st>>>(B.l, P, nmt, L, A.s_ptr, A.s_ent, B.s_ptr,
                                                  B.g_ent, B.g_off, Vals<T>::V(c), C, S,
                                                  c.det ? c.det_buf + 1 : nullptr);
    TB_HIP(hipGetLastError());
}

// opposite-spin term; returns false if this shape needs the direct kernel
template <typename T>
bool launch_ab(Ctx &c, const T *C, T *S, hipStream_t st) {
    switch (slab_ks(c, sizeof(T))) {
        case 4: launch_ab_slab<T, 4>(c, C, S, st); return true;
        case 8: launch_ab_slab<T, 8>(c, C, S, st); return true;
        case 12: launch_ab_slab<T, 12>(c, C, S, st); return true;
        case 16: launch_ab_slab<T, 16>(c, C, S, st); return true;
        case 20: launch_ab_slab<T, 20>(c, C, S, st); return true;
        case 24: launch_ab_slab<T, 24>(c, C, S, st); return true;
        default: break;
    }
    if (!slabg_fits(c)) return false;
    launch_ab_slabg<T>(c, C, S, st);
    return true;
}

// Opposite-spin term, direct double sum (general fallback):
// sigma[I, I'] += sum_{k in L_a(I)} sum_{l in L_b(I')} s_k s_l V[pair_k][pair_l] C[J_k, J'_l]
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ab_direct(int64_t lb, int64_t ncb, int P,
                                                      const int64_t *__restrict__ sa_ptr,
                                                      const Ent *__restrict__ sa_ent,
                                                      const int64_t *__restrict__ sb_ptr,
                                                      const Ent *__restrict__ sb_ent,
                                                      const T *__restrict__ V,
                                                      const T *__restrict__ C, T *__restrict__ S) {
    const int64_t I = blockIdx.x / ncb;
    const int64_t Ip = (blockIdx.x - I * ncb) * kBlock + threadIdx.x;
    if (Ip >= lb) return;
    T acc = 0;
    const int64_t k1 = sa_ptr[I + 1], l0 = sb_ptr[Ip], l1 = sb_ptr[Ip + 1];
    for (int64_t k = sa_ptr[I]; k < k1; ++k) {
        const Ent ea = sa_ent[k];
        const T *Vr = V + (int64_t)(ea.o >> 16) * P;
        const T *Cr = C + (int64_t)ea.j * lb;
        T part = 0;
        for (int64_t l = l0; l < l1; ++l) {
            const Ent eb = sb_ent[l];
            const T t = Vr[eb.o >> 16] * Cr[eb.j];
            part += ((eb.o >> 12) & 1u) ? -t : t;
        }
        acc += ((ea.o >> 12) & 1u) ? -part : part;
    }
    S[I * lb + Ip] += acc;
}

// Deterministic mode: the fixed-point scale of one sigma's opposite-spin
// row.  Every partial sum of an output element is bounded by
// K_a K_b max|V| max|C| (K = longest single-link list of a spin); the scale
// is the power of two that maps that bound just inside 2^62.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_det_absmax(int64_t n, const T *__restrict__ C,
                                                       unsigned long long *__restrict__ out) {
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        m = fmax(m, fabs((double)C[i]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    // non-negative doubles order like their bit patterns
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

__global__ void k_det_scale(double *__restrict__ buf, double bound_per_c) {
    const double maxc = __longlong_as_double((long long)((unsigned long long *)buf)[0]);
    const double b = bound_per_c * maxc;
    int e = 0;
    if (b > 0.0) (void)frexp(b, &e);  // b < 2^e
    buf[1] = ldexp(1.0, 62 - e);
}

template <typename T>
void det_scale(Ctx &c, const T *C, int64_t n, hipStream_t st) {
    const double kb = (double)std::max(c.sp[0].max_s, 1) * (double)std::max(c.sp[1].max_s, 1);
    launch_zero<double>(2, c.det_buf, st);
    const int64_t g = std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 4096));
    k_det_absmax<T><<<(unsigned)g, kBlock, 0, st>>>(n, C, (unsigned long long *)c.det_buf);
    k_det_scale<<<1, 1, 0, st>>>(c.det_buf, kb * c.maxV);
    TB_HIP(hipGetLastError());
}

// sigma with the beta sweep in blocks of rb alpha rows; work holds
// 2 l_beta rb elements of type T (C^T and the sweep result of a block)
template <typename T>
void sigma_impl(Ctx &c, const T *C, T *S, hipStream_t st, int terms, void *work, int64_t rb,
                bool marks, void *hwork, size_t hbytes) {
    const Spin &A = c.sp[0], &B = c.sp[1];
    const int64_t la = A.l, lb = B.l;
    const int prec = sizeof(T) == 8 ? TBSCI_FP64 : TBSCI_FP32;
    auto timing_mark = [&](Ctx &cc, int index, int pr, hipStream_t s2) {
        if (marks) ::tbsci::timing_mark(cc, index, pr, s2);
    };

    // deterministic mode: a problem that can share grouped launches (its
    // beta sweep in one block) sweeps in the grouped sweep's one fixed
    // order; the others are never grouped and keep the panel and chunked
    // sweeps, whose order is fixed too
    const bool fixed = c.det && groupable(c);
    // hole-pair sweeps (with their product buffer; never in the
    // no-allocation entry point)
    const bool ha = hwork && hole_on(c, 0), hb = hwork && hole_on(c, 1);
    timing_mark(c, 0, prec, st);
    if ((terms & 1) && ha)
        hole_sweep(c, 0, lb, C, S, prec, hwork, hbytes, st);  // sigma = A_a C
    else if (terms & 1)
        launch_row_sweep<T>(A, lb, C, S, false, st, fixed);
    else
        launch_zero<T>(la * lb, S, st);
    timing_mark(c, 1, prec, st);
    if (terms & 2) {
        // sigma[r0 : r0 + nr] += (A_b C[r0 : r0 + nr]^T)^T, block by block
        T *Ct = (T *)work, *St = (T *)work + (size_t)lb * rb;
        for (int64_t r0 = 0; r0 < la; r0 += rb) {
            const int64_t nr = std::min(rb, la - r0);
            launch_transpose<T, false>(nr, lb, C + r0 * lb, Ct, st);
            if (hb)
                hole_sweep(c, 1, nr, Ct, St, prec, hwork, hbytes, st);
            else
                launch_row_sweep<T>(B, nr, Ct, St, false, st, fixed);
            launch_transpose<T, true>(lb, nr, St, S + r0 * lb, st);
        }
    }
    timing_mark(c, 2, prec, st);
    if ((terms & 4) && c.det) det_scale(c, C, la * lb, st);
    if (!(terms & 4)) {
    } else if (!launch_ab<T>(c, C, S, st)) {
        const int64_t ncb = (lb + kBlock - 1) / kBlock;
        k_ab_direct<T><<<(unsigned)(la * ncb), kBlock, 0, st>>>(lb, ncb, c.P, A.s_ptr, A.s_ent,
                                                                 B.s_ptr, B.s_ent, Vals<T>::V(c),
                                                                 C, S);
        TB_HIP(hipGetLastError());
    }
    timing_mark(c, 3, prec, st);
}

template <typename T>
void launch_slab_group(const SlabDesc *dd, int nd, int64_t blocks, int P, int KS, size_t lds,
                       Ctx &c0, hipStream_t st) {
    const int nmt = (P + 15) / 16;
    auto f = KS == 4    ? g_ab_slab<T, 4>
             : KS == 8  ? g_ab_slab<T, 8>
             : KS == 12 ? g_ab_slab<T, 12>
             : KS == 16 ? g_ab_slab<T, 16>
             : KS == 20 ? g_ab_slab<T, 20>
             : KS == 24 ? g_ab_slab<T, 24>
                        : nullptr;
    if (!f) throw Error(TBSCI_E_DEVICE, "no grouped slab kernel for this shape");
    if (lds > 64 * 1024) allow_lds(c0, (const void *)f, lds);
    f<<<(unsigned)blocks, kSlabBlock, lds, st>>>(dd, nd, P, nmt);
    TB_HIP(hipGetLastError());
}

template <typename T>
void sigma_group_impl(Ctx *const *ctx, const T *const *C, T *const *S, int n, TableArena &ar,
                      hipStream_t st) {
    std::vector<SweepDesc> sa, sb;
    std::vector<TransDesc> t1, t2;
    int64_t bsa = 0, bsb = 0, bt1 = 0, bt2 = 0;
    auto sweep = [&](std::vector<SweepDesc> &v, int64_t &blk, const Spin &s, int64_t ncols,
                     const T *X, T *Y) {
        const int vec = sweep_vec_of<T>(ncols);
        const int64_t ntiles = (ncols + 64 * vec - 1) / (64 * vec), nrb = (s.l + 3) / 4;
        const int64_t tpx = (ntiles + kXcd - 1) / kXcd;
        v.push_back(SweepDesc{blk, s.l, ncols, ntiles, nrb, tpx, s.a_ptr, s.a_col, Vals<T>::a(s),
                              X, Y});
        blk += kXcd * tpx * nrb;  // a multiple of 8
    };
    auto trans = [&](std::vector<TransDesc> &v, int64_t &blk, int64_t R, int64_t Cn, const T *in,
                     T *out) {
        const int64_t ntr = (R + 31) / 32, ntc = (Cn + 31) / 32;
        v.push_back(TransDesc{blk, R, Cn, ntc, in, out});
        blk += ntr * ntc;
    };
    struct SlabGroup {
        int P, KS;
        size_t lds;
        int64_t blocks;
        std::vector<SlabDesc> d;
    };
    std::vector<SlabGroup> sgroups;
    std::vector<int> direct;
    for (int i = 0; i < n; ++i) {
        Ctx &c = *ctx[i];
        const Spin &A = c.sp[0], &B = c.sp[1];
        T *Ct = (T *)ctx_workspace(c), *St = Ct + (size_t)A.l * B.l;
        if (c.det) det_scale(c, C[i], A.l * B.l, st);
        sweep(sa, bsa, A, B.l, C[i], S[i]);
        trans(t1, bt1, A.l, B.l, C[i], Ct);
        sweep(sb, bsb, B, A.l, Ct, St);
        trans(t2, bt2, B.l, A.l, St, S[i]);
        const int SK = slab_ks(c, sizeof(T));
        if (SK) {  // slab kernel; problems with the same P and KS share a launch
            const SlabLds L =
                slab_lds(B.l, (c.P + 15) / 16, std::max((A.max_s + 3) / 4, 1), sizeof(T));
            SlabGroup *g = nullptr;
            for (auto &x : sgroups)
                if (x.P == c.P && x.KS == SK) g = &x;
            if (!g) {
                sgroups.push_back(SlabGroup{c.P, SK, 0, 0, {}});
                g = &sgroups.back();
            }
            g->d.push_back(SlabDesc{g->blocks, B.l, L, A.s_ptr, A.s_ent, B.s_ptr, B.g_ent,
                                    B.g_off, Vals<T>::V(c), C[i], S[i],
                                    c.det ? c.det_buf + 1 : nullptr});
            g->blocks += A.l;
            g->lds = std::max(g->lds, L.total);
            continue;
        }
        direct.push_back(i);  // single-problem opposite-spin kernel
    }
    if (n == 0) return;
    const SweepDesc *dsa = ar.stage(sa.data(), sa.size());
    const SweepDesc *dsb = ar.stage(sb.data(), sb.size());
    const TransDesc *dt1 = ar.stage(t1.data(), t1.size());
    const TransDesc *dt2 = ar.stage(t2.data(), t2.size());
    std::vector<const SlabDesc *> dsg;
    for (auto &g : sgroups) dsg.push_back(ar.stage(g.d.data(), g.d.size()));
    ar.flush(st);
    g_row_sweep<T, false><<<(unsigned)bsa, kBlock, 0, st>>>(dsa, n);  // sigma = A_a C
    g_transpose<T, false><<<(unsigned)bt1, kBlock, 0, st>>>(dt1, n);
    g_row_sweep<T, false><<<(unsigned)bsb, kBlock, 0, st>>>(dsb, n);
    g_transpose<T, true><<<(unsigned)bt2, kBlock, 0, st>>>(dt2, n);  // sigma += (A_b C^T)^T
    TB_HIP(hipGetLastError());
    for (size_t k = 0; k < sgroups.size(); ++k)
        launch_slab_group<T>(dsg[k], (int)sgroups[k].d.size(), sgroups[k].blocks, sgroups[k].P,
                             sgroups[k].KS, sgroups[k].lds, *ctx[0], st);
    for (int i : direct) {  // single-problem opposite-spin kernels
        Ctx &c = *ctx[i];
        if (launch_ab<T>(c, C[i], S[i], st)) continue;
        const Spin &A = c.sp[0], &B = c.sp[1];
        const int64_t ncb = (B.l + kBlock - 1) / kBlock;
        k_ab_direct<T><<<(unsigned)(A.l * ncb), kBlock, 0, st>>>(B.l, ncb, c.P, A.s_ptr, A.s_ent,
                                                                  B.s_ptr, B.s_ent, Vals<T>::V(c),
                                                                  C[i], S[i]);
        TB_HIP(hipGetLastError());
    }
}

}  // namespace

// entries of the fixed-point staging area that deterministic sigma needs:
// the part of each alpha row beyond the LDS row of the global-fragment
// kernel (0 when whole rows fit, or another kernel takes the shape)
int64_t det_stage_entries(const Ctx &c) {
    if (!slabg_fits(c)) return 0;
    const Spin &A = c.sp[0], &B = c.sp[1];
    const int ks = std::max((A.max_s + 3) / 4, 1);
    const SlabgLds L = slabg_lds(B.l, ks, 8);
    return L.nrow < B.l ? A.l * (B.l - L.nrow) : 0;
}

void launch_sigma_group(Ctx *const *ctx, const void *const *C, void *const *S, int n,
                        int precision, TableArena &ar, hipStream_t st) {
    // problems whose beta sweep runs in more than one block take their own
    // launches; the others share them.  A context that appears again (the
    // two spin-flip sectors of one problem) shares its beta-sweep workspace,
    // so its later appearances run after the shared launches, in stream order
    std::vector<Ctx *> gc;
    std::vector<const void *> gC;
    std::vector<void *> gS;
    std::vector<int> later;
    for (int i = 0; i < n; ++i) {
        if (n == 1 || !groupable(*ctx[i])) {
            launch_sigma(*ctx[i], C[i], S[i], precision, st);
        } else if (std::find(gc.begin(), gc.end(), ctx[i]) != gc.end()) {
            later.push_back(i);
        } else {
            gc.push_back(ctx[i]);
            gC.push_back(C[i]);
            gS.push_back(S[i]);
        }
    }
    const int m = (int)gc.size();
    if (m == 1) {
        launch_sigma(*gc[0], gC[0], gS[0], precision, st);
    } else if (m > 1) {
        if (precision == TBSCI_FP64)
            sigma_group_impl<double>(gc.data(), (const double *const *)gC.data(),
                                     (double *const *)gS.data(), m, ar, st);
        else
            sigma_group_impl<float>(gc.data(), (const float *const *)gC.data(),
                                    (float *const *)gS.data(), m, ar, st);
    }
    for (int i : later) launch_sigma(*ctx[i], C[i], S[i], precision, st);
}

void reserve_sigma_workspace(Ctx &c) {
    (void)ctx_workspace(c);
    if (hole_any(c)) (void)hole_workspace(c);
}

void timing_mark(Ctx &c, int index, int precision, hipStream_t st) {
    if (!c.timing) return;
    if (index == 0) {
        Ctx::TimedCall t{};
        t.precision = precision;
        for (auto &e : t.ev) TB_HIP(hipEventCreate(&e));
        c.timed.push_back(t);
    }
    TB_HIP(hipEventRecord(c.timed.back().ev[index], st));
}

void timing_clear(Ctx &c) {
    for (auto &t : c.timed)
        for (auto &e : t.ev)
            if (e) (void)hipEventDestroy(e);
    c.timed.clear();
}

void launch_sigma_ws(Ctx &c, const void *C, void *S, int precision, hipStream_t st, int terms,
                     void *work, size_t work_bytes, bool marks, void *hwork, size_t hbytes) {
    const int64_t la = c.sp[0].l, lb = c.sp[1].l;
    int64_t rb = la;
    if (terms & 2) {
        rb = beta_block_rows(la, lb, work_bytes);
        if (rb < 1)
            throw Error(TBSCI_E_INVAL, "the workspace cannot hold the beta sweep of one alpha row");
    }
    if (precision == TBSCI_FP64)
        sigma_impl<double>(c, (const double *)C, (double *)S, st, terms, work, rb, marks, hwork,
                           hbytes);
    else
        sigma_impl<float>(c, (const float *)C, (float *)S, st, terms, work, rb, marks, hwork,
                          hbytes);
}

void launch_sigma(Ctx &c, const void *C, void *S, int precision, hipStream_t st, int terms) {
    void *w = ctx_workspace(c);
    void *hw = hole_any(c) ? hole_workspace(c) : nullptr;
    launch_sigma_ws(c, C, S, precision, st, terms, w, c.work_bytes, true, hw,
                    hw ? c.hole_work_bytes : 0);
}

// Floating-point operations one launch of kernel `kernel` executes: for the
// MFMA opposite-spin kernels the padded tiles (K rounded up to the 4-deep
// k-step, or to chunks of 4 k-steps in the FP32 slab kernel; pairs to
// 16-row M-tiles; beta columns to 16-column slabs); for the sweeps and the
// direct fallback the multiply-adds of their sums.
double executed_flops(Ctx &c, int kernel, int precision) {
    const Spin &A = c.sp[0], &B = c.sp[1];
    // hole-pair sweeps: each hole string's padded product block times the
    // columns, rounded up to the 16-column MFMA tile
    if (kernel == 0 && hole_on(c, 0)) return 2.0 * A.hole_mfma * (double)((B.l + 15) / 16 * 16);
    if (kernel == 1 && hole_on(c, 1)) return 2.0 * B.hole_mfma * (double)((A.l + 15) / 16 * 16);
    if (kernel == 0) return 2.0 * (double)A.n_a * (double)B.l;
    if (kernel == 1) return 2.0 * (double)B.n_a * (double)A.l;
    const int nmt = (c.P + 15) / 16;
    const bool slab = slab_ks(c, precision == TBSCI_FP32 ? sizeof(float) : sizeof(double)) > 0;
    if (!slab && !slabg_fits(c)) return 2.0 * (double)A.n_s * (double)B.n_s;
    const double cols = (double)((B.l + 15) / 16) * 16;
    double kp = 0.0;
    if (!slab) {
        // global-fragment kernel: every row of a class runs the class's k-steps
        static const int kcls[5] = {8, 16, 24, 28, 32};
        for (int k = 0; k < 5; ++k) kp += 4.0 * kcls[k] * (double)(A.ks_off[k + 1] - A.ks_off[k]);
        return 2.0 * kp * (16.0 * nmt) * cols;
    }
    std::vector<int64_t> ptr((size_t)A.l + 1);
    TB_HIP(hipMemcpy(ptr.data(), A.s_ptr, ptr.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    const int64_t pad = precision == TBSCI_FP32 ? 16 : 4;
    for (int64_t i = 0; i < A.l; ++i)
        kp += (double)(pad * ((ptr[i + 1] - ptr[i] + pad - 1) / pad));
    return 2.0 * kp * (16.0 * nmt) * cols;
}

}  // namespace tbsci
