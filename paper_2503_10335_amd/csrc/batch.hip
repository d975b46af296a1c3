// Davidson solver engine (grouped vector kernels, the round scheduler) and
// the C entry points tbsci_davidson, tbsci_davidson_batch and
// tbsci_sigma_batch.  The iteration is Davidson on the sigma product (paper
// Sec. II.B), with a bounded restart (Sec. III.C: the stored vectors stay
// bounded by the subspace size) and, in mixed precision, a single-precision
// sigma with everything else in double precision (Sec. III.A).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "batch.hpp"

namespace tbsci {

void jacobi_eigh(int k, std::vector<double> A, std::vector<double> &w, std::vector<double> &Z);

namespace {

constexpr int kB = 256;
constexpr int kSV = kBatchMaxVec;
constexpr int kNbMax = 2048;
// scalar area of a slot (doubles)
constexpr int sCol = 0;         // [kSV] V_i . W_new
constexpr int sR2 = kSV;        // |r|^2 of the round's Ritz pair
constexpr int sTn2 = kSV + 2;   // |t|^2 after Gram-Schmidt
constexpr int sN2 = kSV + 3;    // |previous direction|^2 after re-orthogonalisation
constexpr int sG = kSV + 4;     // x.Wx, x.Wxp, xp.Wx, xp.Wxp
constexpr int sArg = kSV + 8;   // start index
constexpr int sGN = kSV + 9;    // |guess|^2
constexpr int sSign = kSV + 10; // sign of the output vector
constexpr int sRO = kSV + 11;   // re-orthogonalisation coefficient
constexpr int sD1 = 2 * kSV;    // [kSV] first-pass coefficients, then |t|^2
constexpr int sD2 = 3 * kSV;    // [kSV] second-pass coefficients
constexpr int kScal = 4 * kSV;  // row length

// One slot's part of a grouped launch.  Grid-stride kernels give slot d the
// blocks [blk0, blk0 + nb); the reduce and per-slot kernels index d directly.
struct VDesc {
    int64_t blk0, n;
    int32_t nb, k;
    int32_t dst, src, src2;  // scalar-area indices
    int32_t flip;
    double thresh;
    double *o0, *o1, *o2;
    const double *in;
    float *f;
    double *partial, *scal;
    const double *a[kSV];
    const double *b[kSV];
    double c[kSV];
    double theta, floor_;
    int64_t lb;
    int32_t M, pad;
    const uint64_t *astr;
    const double *da, *db, *jb;
    const uint32_t *mask;  // TBSCI space: kept determinants (bit u of row w), else null
    int64_t wpr;
};

// whether determinant t of a slot's zero-extended layout belongs to its space
__device__ __forceinline__ bool kept(const VDesc &e, int64_t t) {
    if (!e.mask) return true;
    const int64_t w = t / e.lb, u = t - w * e.lb;
    return (e.mask[w * e.wpr + (u >> 5)] >> (u & 31)) & 1u;
}

__device__ __forceinline__ const VDesc &slot_of(const VDesc *__restrict__ d, int nd, int64_t &lblk) {
    int lo = 0, hi = nd - 1;
    const int64_t b = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].blk0 <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    lblk = b - d[lo].blk0;
    return d[lo];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// out[i * kNbMax] = block sum of acc[i], i < k (fixed order: deterministic)
__device__ __forceinline__ void block_sums(const double (&acc)[kSV], int k, double *out) {
    __shared__ double red[kB / 64][kSV];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < kSV; ++i)
        if (i < k) {
            const double s = wave_sum(acc[i]);
            if (l == 0) red[w][i] = s;
        }
    __syncthreads();
    if ((int)threadIdx.x < k) {
        double s = 0.0;
#pragma unroll
        for (int ww = 0; ww < kB / 64; ++ww) s += red[ww][threadIdx.x];
        out[threadIdx.x * kNbMax] = s;
    }
    __syncthreads();
}

#define TB_SLOT_LOOP(e, lblk, t) \
    for (int64_t t = lblk * kB + threadIdx.x; t < e.n; t += (int64_t)e.nb * kB)

// Kernels over the k vectors of a basis run a body templated on k, so that
// each element's k loads are issued together (a loop guarded by i < k
// issues them one branch at a time).  The arithmetic order is that of a
// loop over i ascending.
#define TB_K_DISPATCH(k, CALL)                                                            \
    switch (k) {                                                                         \
        case 1: CALL(1); break;   case 2: CALL(2); break;   case 3: CALL(3); break;      \
        case 4: CALL(4); break;   case 5: CALL(5); break;   case 6: CALL(6); break;      \
        case 7: CALL(7); break;   case 8: CALL(8); break;   case 9: CALL(9); break;      \
        case 10: CALL(10); break; case 11: CALL(11); break; case 12: CALL(12); break;    \
        case 13: CALL(13); break; case 14: CALL(14); break; case 15: CALL(15); break;    \
        case 16: CALL(16); break; default: break;                                        \
    }
static_assert(kSV == 16, "TB_K_DISPATCH covers k = 1 .. 16");

// H_KK from the per-string parts
__device__ __forceinline__ double diag_at(const VDesc &e, int64_t t) {
    const int64_t ia = t / e.lb, ib = t - ia * e.lb;
    double d = e.da[ia] + e.db[ib];
    const double *jr = e.jb + ib * e.M;
    for (uint64_t m = e.astr[ia]; m; m &= m - 1) d += jr[__builtin_ctzll(m)];
    return d;
}

// (value, index) pair reduction over the block: smallest (MIN) or largest
// value, first index on ties; every thread receives the result
template <bool MIN>
__device__ __forceinline__ void block_pick(double v, int64_t i, double *pv, int64_t *pi) {
    __shared__ double sv[kB];
    __shared__ int64_t si[kB];
    sv[threadIdx.x] = v;
    si[threadIdx.x] = i;
    __syncthreads();
    for (int off = kB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            const double v2 = sv[threadIdx.x + off];
            const int64_t i2 = si[threadIdx.x + off];
            const double v1 = sv[threadIdx.x];
            const int64_t i1 = si[threadIdx.x];
            const bool better = MIN ? v2 < v1 : v2 > v1;
            if (i2 >= 0 && (i1 < 0 || better || (v2 == v1 && i2 < i1))) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    *pv = sv[0];
    *pi = si[0];
    __syncthreads();
}

__global__ __launch_bounds__(kB) void gv_fill(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    TB_SLOT_LOOP(e, lb, t) e.o0[t] = 0.0;
}

__global__ __launch_bounds__(kB) void gv_copy(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    TB_SLOT_LOOP(e, lb, t) e.o0[t] = e.in[t];
}

// per block: smallest H_KK and its first index (in the antisymmetric
// sector of a flip-symmetric space only open-shell determinants I != J)
__global__ __launch_bounds__(kB) void gv_diag_min(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    double best = 1e308;
    int64_t bi = -1;
    TB_SLOT_LOOP(e, lb, t) {
        if (e.flip < 0 && t / e.lb == t % e.lb) continue;
        if (!kept(e, t)) continue;
        const double v = diag_at(e, t);
        if (v < best) {
            best = v;
            bi = t;
        }
    }
    double pv;
    int64_t pi;
    block_pick<true>(best, bi, &pv, &pi);
    if (threadIdx.x == 0) {
        e.partial[lb] = pv;
        e.partial[kNbMax + lb] = (double)pi;
    }
}

// one block per slot: the start vector is the unit vector on the smallest
// H_KK (first on ties); in a flip-symmetric space an open-shell |I J> is
// paired with |J I>: (|I J> + flip |J I>)/sqrt 2 for sector flip = +1 or -1
__global__ __launch_bounds__(kB) void gv_argmin_unit(const VDesc *__restrict__ d) {
    const VDesc e = d[blockIdx.x];
    double best = 1e308;
    int64_t bi = -1;
    for (int b = threadIdx.x; b < e.nb; b += kB) {
        const double v = e.partial[b];
        const int64_t i = (int64_t)e.partial[kNbMax + b];
        if (i >= 0 && (bi < 0 || v < best || (v == best && i < bi))) {
            best = v;
            bi = i;
        }
    }
    double pv;
    int64_t pi;
    block_pick<true>(best, bi, &pv, &pi);
    if (threadIdx.x == 0) {
        const int64_t at = pi >= 0 ? pi : 0;
        const int64_t ia = at / e.lb, ib = at - ia * e.lb;
        const int64_t at2 = e.flip ? ib * e.lb + ia : at;
        const double val = at2 == at ? 1.0 : 0.70710678118654752440;
        e.o0[at2] = e.flip < 0 ? -val : val;
        e.o0[at] = val;
        e.scal[e.dst] = (double)at;
    }
}

// per block: largest |x| and its first index
__global__ __launch_bounds__(kB) void gv_absmax(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    double best = -1.0;
    int64_t bi = -1;
    TB_SLOT_LOOP(e, lb, t) {
        const double v = fabs(e.in[t]);
        if (v > best) {
            best = v;
            bi = t;
        }
    }
    double pv;
    int64_t pi;
    block_pick<false>(best, bi, &pv, &pi);
    if (threadIdx.x == 0) {
        e.partial[lb] = pv;
        e.partial[kNbMax + lb] = (double)pi;
    }
}

// one block per slot: the sign that makes the largest-magnitude entry
// positive
__global__ __launch_bounds__(kB) void gv_absmax_sign(const VDesc *__restrict__ d) {
    const VDesc e = d[blockIdx.x];
    double best = -1.0;
    int64_t bi = -1;
    for (int b = threadIdx.x; b < e.nb; b += kB) {
        const double v = e.partial[b];
        const int64_t i = (int64_t)e.partial[kNbMax + b];
        if (i >= 0 && (bi < 0 || v > best || (v == best && i < bi))) {
            best = v;
            bi = i;
        }
    }
    double pv;
    int64_t pi;
    block_pick<false>(best, bi, &pv, &pi);
    if (threadIdx.x == 0) e.scal[e.dst] = (pi >= 0 && e.in[pi] < 0.0) ? -1.0 : 1.0;
}

__global__ __launch_bounds__(kB) void gv_signed_copy(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    const double s = e.scal[e.src];
    TB_SLOT_LOOP(e, lb, t) e.o0[t] = s * e.in[t];
}

// o0 = H_KK for every determinant of the slot (stored for the whole solve)
__global__ __launch_bounds__(kB) void gv_diag(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    TB_SLOT_LOOP(e, lb, t) e.o0[t] = diag_at(e, t);
}

// x = V y, wx = W y, t = (wx - theta x) / (theta - H_KK) with a floor;
// partial sums of |wx - theta x|^2 (H_KK read from the stored diagonal)
template <int K>
__device__ __forceinline__ void ritz_body(const VDesc &e, int64_t lb, double *acc) {
    TB_SLOT_LOOP(e, lb, t) {
        double av[K], bv[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            av[i] = e.a[i][t];
            bv[i] = e.b[i][t];
        }
        const double dk = e.in ? e.in[t] : diag_at(e, t);
        double xv = 0.0, wv = 0.0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            xv += e.c[i] * av[i];
            wv += e.c[i] * bv[i];
        }
        const double r = wv - e.theta * xv;
        acc[0] += r * r;
        double den = e.theta - dk;
        if (fabs(den) < e.floor_) den = den < 0.0 ? -e.floor_ : e.floor_;
        e.o0[t] = xv;
        e.o1[t] = wv;
        e.o2[t] = r / den;
    }
}

__global__ __launch_bounds__(kB) void gv_ritz(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    double acc[kSV] = {};
    if (e.k == 0) {  // empty basis: zero vectors
        TB_SLOT_LOOP(e, lb, t) e.o0[t] = e.o1[t] = e.o2[t] = 0.0;
    }
#define TB_CALL(K) ritz_body<K>(e, lb, acc)
    TB_K_DISPATCH(e.k, TB_CALL)
#undef TB_CALL
    block_sums(acc, 1, e.partial + lb);
}

// o0 = sum_i c_i a_i, o1 = sum_i c_i b_i
template <int K>
__device__ __forceinline__ void lincomb2_body(const VDesc &e, int64_t lb) {
    TB_SLOT_LOOP(e, lb, t) {
        double av[K], bv[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            av[i] = e.a[i][t];
            bv[i] = e.b[i][t];
        }
        double xv = 0.0, wv = 0.0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            xv += e.c[i] * av[i];
            wv += e.c[i] * bv[i];
        }
        e.o0[t] = xv;
        e.o1[t] = wv;
    }
}

__global__ __launch_bounds__(kB) void gv_lincomb2(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    if (e.k == 0) {  // empty basis: zero vectors
        TB_SLOT_LOOP(e, lb, t) e.o0[t] = e.o1[t] = 0.0;
    }
#define TB_CALL(K) lincomb2_body<K>(e, lb)
    TB_K_DISPATCH(e.k, TB_CALL)
#undef TB_CALL
}

// partial[i][blk] = block's part of a_i . in, i < k, with `in` read once
template <int K>
__device__ __forceinline__ void dots_body(const VDesc &e, int64_t lb, double *acc) {
    TB_SLOT_LOOP(e, lb, t) {
        double av[K];
#pragma unroll
        for (int i = 0; i < K; ++i) av[i] = e.a[i][t];
        const double x = e.in[t];
#pragma unroll
        for (int i = 0; i < K; ++i) acc[i] += av[i] * x;
    }
}

__global__ __launch_bounds__(kB) void gv_dots(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    double acc[kSV] = {};
#define TB_CALL(K) dots_body<K>(e, lb, acc)
    TB_K_DISPATCH(e.k, TB_CALL)
#undef TB_CALL
    block_sums(acc, e.k, e.partial + lb);
}

// o0 -= sum_i scal[src + i] a_i, then partial[i][blk] = a_i . o0: the
// subtraction of the first Gram-Schmidt pass with the dot products of the
// second
template <int K>
__device__ __forceinline__ void subdots_body(const VDesc &e, int64_t lb, const double *cf,
                                             double *acc) {
    TB_SLOT_LOOP(e, lb, t) {
        double av[K];
#pragma unroll
        for (int i = 0; i < K; ++i) av[i] = e.a[i][t];
        double v = e.o0[t];
#pragma unroll
        for (int i = 0; i < K; ++i) v -= cf[i] * av[i];
        e.o0[t] = v;
#pragma unroll
        for (int i = 0; i < K; ++i) acc[i] += av[i] * v;
    }
}

__global__ __launch_bounds__(kB) void gv_subdots(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    double cf[kSV], acc[kSV] = {};
#pragma unroll
    for (int i = 0; i < kSV; ++i) cf[i] = i < e.k ? e.scal[e.src + i] : 0.0;
#define TB_CALL(K) subdots_body<K>(e, lb, cf, acc)
    TB_K_DISPATCH(e.k, TB_CALL)
#undef TB_CALL
    block_sums(acc, e.k, e.partial + lb);
}

// o0 -= sum_i scal[src + i] a_i, then partial[0][blk] = |o0|^2
template <int K>
__device__ __forceinline__ void subnorm_body(const VDesc &e, int64_t lb, const double *cf,
                                             double *acc) {
    TB_SLOT_LOOP(e, lb, t) {
        double av[K];
#pragma unroll
        for (int i = 0; i < K; ++i) av[i] = e.a[i][t];
        double v = e.o0[t];
#pragma unroll
        for (int i = 0; i < K; ++i) v -= cf[i] * av[i];
        e.o0[t] = v;
        acc[0] += v * v;
    }
}

__global__ __launch_bounds__(kB) void gv_subnorm(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    double cf[kSV], acc[kSV] = {};
#pragma unroll
    for (int i = 0; i < kSV; ++i) cf[i] = i < e.k ? e.scal[e.src + i] : 0.0;
    if (e.k == 0) {  // |o0|^2 alone
        TB_SLOT_LOOP(e, lb, t) {
            const double v = e.o0[t];
            acc[0] += v * v;
        }
    }
#define TB_CALL(K) subnorm_body<K>(e, lb, cf, acc)
    TB_K_DISPATCH(e.k, TB_CALL)
#undef TB_CALL
    block_sums(acc, 1, e.partial + lb);
}

// scal[dst + i] = sum over the slot's blocks of partial[i][.]; block = (slot, i)
__global__ __launch_bounds__(kB) void gv_reduce(const VDesc *__restrict__ d, int kmax) {
    __shared__ double red[kB];
    const VDesc e = d[blockIdx.x / kmax];
    const int i = blockIdx.x % kmax;
    if (i >= e.k) return;
    double s = 0.0;
    for (int b = threadIdx.x; b < e.nb; b += kB) s += e.partial[i * kNbMax + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = kB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) e.scal[e.dst + i] = red[0];
}

// o0 -= sum_i scal[src + i] a_i (and o1 -= sum_i scal[src + i] b_i)
template <int K>
__device__ __forceinline__ void subproj_body(const VDesc &e, int64_t lb, const double *cf) {
    TB_SLOT_LOOP(e, lb, t) {
        double av[K];
#pragma unroll
        for (int i = 0; i < K; ++i) av[i] = e.a[i][t];
        double v = e.o0[t];
#pragma unroll
        for (int i = 0; i < K; ++i) v -= cf[i] * av[i];
        e.o0[t] = v;
        if (e.o1) {
            double bv[K];
#pragma unroll
            for (int i = 0; i < K; ++i) bv[i] = e.b[i][t];
            double w = e.o1[t];
#pragma unroll
            for (int i = 0; i < K; ++i) w -= cf[i] * bv[i];
            e.o1[t] = w;
        }
    }
}

__global__ __launch_bounds__(kB) void gv_subproj(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    double cf[kSV];
#pragma unroll
    for (int i = 0; i < kSV; ++i) cf[i] = i < e.k ? e.scal[e.src + i] : 0.0;
#define TB_CALL(K) subproj_body<K>(e, lb, cf)
    TB_K_DISPATCH(e.k, TB_CALL)
#undef TB_CALL
}

// o0 (and o1) *= 1 / |.| with |.| = sqrt(scal[src]), or by 0 when |.| <=
// thresh (times sqrt(scal[src2]) when src2 >= 0: a relative test)
__global__ __launch_bounds__(kB) void gv_scale(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    const double nrm = sqrt(fmax(e.scal[e.src], 0.0));
    const double ref = e.src2 >= 0 ? sqrt(fmax(e.scal[e.src2], 0.0)) : 1.0;
    const double f = nrm > e.thresh * ref ? 1.0 / nrm : 0.0;
    TB_SLOT_LOOP(e, lb, t) {
        e.o0[t] *= f;
        if (e.o1) e.o1[t] *= f;
    }
}

// correction vectors of flip-symmetric slots: T = (T + flip T^T) / 2; d.nb
// is the slot's tile-pair block count here
__global__ __launch_bounds__(kB) void gv_flip_sym(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    flip_sym_block(lb, e.lb, (double)e.flip, e.o0);
}

// zero the entries of o0 outside the slot's TBSCI space
__global__ __launch_bounds__(kB) void gv_mask(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    TB_SLOT_LOOP(e, lb, t) if (!kept(e, t)) e.o0[t] = 0.0;
}

__global__ __launch_bounds__(kB) void gv_to_f32(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    TB_SLOT_LOOP(e, lb, t) e.f[t] = (float)e.in[t];
}

__global__ __launch_bounds__(kB) void gv_to_f64(const VDesc *__restrict__ d, int nd) {
    int64_t lb;
    const VDesc e = slot_of(d, nd, lb);
    TB_SLOT_LOOP(e, lb, t) e.o0[t] = (double)e.f[t];
}

#undef TB_SLOT_LOOP

// operations of a round, in issue order (a slot uses a subsequence)
enum Op {
    O_AMAX, O_AMAX_S, O_OUT,                        // finish: signed copy to the output
    O_DIAG,                                         // start: the stored diagonal
    O_FILL, O_DMIN, O_AMIN,                         // start on the smallest H_KK
    O_GCOPY, O_GN_D, O_GN_R, O_GN_S,                // start from a guess
    O_RITZ, O_RITZ_R, O_SYM,                        // Ritz pair, residual, correction
    O_LC, O_RO1_D, O_RO1_R, O_RO1_S, O_RO2_D, O_RO2_R, O_RO2_S,  // restart
    O_N2_D, O_N2_R, O_N2_S, O_G0_D, O_G0_R, O_G1_D, O_G1_R,
    O_D1, O_D1_R, O_S1D2, O_S1D2_R, O_S2N, O_S2N_R, O_TSCALE,    // Gram-Schmidt
    O_CVT32,
    O_SIGMA,  // marker: grouped sigma builds
    O_CVT64,
    O_MASK,                                         // TBSCI space: sigma restricted to it
    O_COL_D, O_COL_R,                               // new column of V^T H V
    O_N
};

enum Kind {
    K_DIAG, K_FILL, K_COPY, K_DMIN, K_AMIN, K_AMAX, K_ASIGN, K_SCOPY, K_RITZ, K_RED, K_SYM, K_LC,
    K_DOT, K_SUB, K_SUBDOT, K_SUBNORM, K_SCALE, K_F32, K_F64, K_MASK, K_NONE
};

Kind kind_of(int op) {
    switch (op) {
        case O_AMAX: return K_AMAX;
        case O_AMAX_S: return K_ASIGN;
        case O_OUT: return K_SCOPY;
        case O_DIAG: return K_DIAG;
        case O_FILL: return K_FILL;
        case O_DMIN: return K_DMIN;
        case O_AMIN: return K_AMIN;
        case O_GCOPY: return K_COPY;
        case O_RITZ: return K_RITZ;
        case O_SYM: return K_SYM;
        case O_LC: return K_LC;
        case O_RO1_S: case O_RO2_S: return K_SUB;
        case O_S1D2: return K_SUBDOT;
        case O_S2N: return K_SUBNORM;
        case O_GN_S: case O_N2_S: case O_TSCALE: return K_SCALE;
        case O_CVT32: return K_F32;
        case O_CVT64: return K_F64;
        case O_MASK: return K_MASK;
        case O_SIGMA: return K_NONE;
        case O_GN_R: case O_RITZ_R: case O_RO1_R: case O_RO2_R: case O_N2_R: case O_G0_R:
        case O_G1_R: case O_D1_R: case O_S1D2_R: case O_S2N_R: case O_COL_R: return K_RED;
        default: return K_DOT;
    }
}

int blocks_for_slot(int64_t n) {
    return (int)std::min<int64_t>(kNbMax, std::max<int64_t>(1, (n + 16 * kB - 1) / (16 * kB)));
}

size_t page(size_t bytes) { return (std::max<size_t>(bytes, 8) + 4095) & ~size_t(4095); }

}  // namespace

struct BatchEngine::Stage {
    std::vector<VDesc> ops[O_N];
    std::vector<Ctx *> c64, c32;
    std::vector<const void *> i64, i32;
    std::vector<void *> o64, o32;
};

BatchEngine::BatchEngine(int device, hipStream_t st) : device_(device), st_(st), ar_(8u << 20) {
    TB_HIP(hipMalloc((void **)&scal_dev_, sizeof(double) * kScal * kBatchMaxSlots));
    TB_HIP(hipHostMalloc((void **)&scal_host_, sizeof(double) * kScal * kBatchMaxSlots,
                         hipHostMallocDefault));
    TB_HIP(hipEventCreate(&ev_[0]));
    TB_HIP(hipEventCreate(&ev_[1]));
    for (int r = kBatchMaxSlots - 1; r >= 0; --r) free_rows_.push_back(r);
}

BatchEngine::~BatchEngine() {
    for (auto &e : ev_)
        if (e) (void)hipEventDestroy(e);
    if (scal_dev_) (void)hipFree(scal_dev_);
    if (scal_host_) (void)hipHostFree(scal_host_);
}

size_t BatchEngine::slot_bytes(int64_t n, const tbsci_davidson_opts &o, bool lean) {
    const size_t v = page(8 * (size_t)n);
    // full: V and W pools of n_max + 3 and the stored diagonal; lean: pools
    // of n_max + 2 and n_max + 1, the diagonal recomputed
    const size_t nvec = lean ? 2 * (size_t)o.n_max + 3 : 2 * (size_t)(o.n_max + 3) + 1;
    size_t b = nvec * v + page(8 * (size_t)kSV * kNbMax);
    if (o.precision == TBSCI_MIXED) b += 2 * page(4 * (size_t)n);
    return b;
}

BatchSlot *BatchEngine::make_slot(Ctx *c, const tbsci_davidson_opts &o, bool guess, bool split) {
    const int64_t n = c->sp[0].l * c->sp[1].l;
    bool lean = o.storage == TBSCI_STORE_LEAN;
    if (o.storage == TBSCI_STORE_AUTO) {
        size_t fr = 0, tot = 0;
        TB_HIP(hipSetDevice(c->device));
        TB_HIP(hipMemGetInfo(&fr, &tot));
        lean = (double)slot_bytes(n, o, false) > 0.9 * (double)fr;
    }
    // sectors: a flip-symmetric space without a start vector is solved in
    // the sector asked for, or in both (symmetric first)
    int sector = 0, npass = 1;
    if (c->flip && !guess) {
        const bool anti_empty = c->sp[0].l < 2 || (c->dets && !c->dets->open_pairs);
        if (o.sector == -1 && anti_empty)
            throw Error(TBSCI_E_INVAL, "the antisymmetric sector of this space is empty");
        sector = o.sector != 0 ? o.sector : 1;
        npass = (o.sector == 0 && !anti_empty) ? 2 : 1;
    }
    auto *s = new BatchSlot();
    try {
        s->c = c;
        s->o = o;
        s->n = n;
        s->nb = blocks_for_slot(s->n);
        s->sector = sector;
        s->npass = npass;
        s->lean = lean;
        auto get = [&](size_t bytes) {
            void *p = nullptr;
            TB_HIP(hipMalloc(&p, bytes));
            s->all.push_back((double *)p);
            s->bytes += page(bytes);
            return p;
        };
        const int nv = lean ? o.n_max + 2 : o.n_max + 3, nw = lean ? o.n_max + 1 : o.n_max + 3;
        for (int i = 0; i < nv; ++i) s->vfree.push_back((double *)get(8 * (size_t)s->n));
        for (int i = 0; i < nw; ++i) s->wfree.push_back((double *)get(8 * (size_t)s->n));
        if (!lean) s->diag = (double *)get(8 * (size_t)s->n);
        s->partial = (double *)get(8 * (size_t)kSV * kNbMax);
        if (o.precision == TBSCI_MIXED) {
            s->f32a = (float *)get(4 * (size_t)s->n);
            s->f32b = (float *)get(4 * (size_t)s->n);
        }
        s->G.assign((size_t)o.n_max * o.n_max, 0.0);
        if (split && npass == 2) {  // the antisymmetric sector in a slot of its own
            tbsci_davidson_opts ot = o;
            ot.sector = -1;
            ot.storage = lean ? TBSCI_STORE_LEAN : TBSCI_STORE_FULL;
            s->twin = make_slot(c, ot, false, false);
            s->twin->primary = s;
            s->npass = 1;
            s->bytes += s->twin->bytes;
        }
    } catch (...) {
        free_slot(s);
        throw;
    }
    return s;
}

void BatchEngine::free_slot(BatchSlot *s) {
    if (!s) return;
    if (s->twin) free_slot(s->twin);
    for (double *p : s->all)
        if (p) (void)hipFree(p);
    delete s;
}

void BatchEngine::add(BatchSlot *s) {
    if (s->twin) {
        if (free_rows_.size() < 2) throw Error(TBSCI_E_STATE, "batch is full");
        s->twin->user = s->user;
        add(s->twin);
    }
    s->held = false;
    if (free_rows_.empty()) throw Error(TBSCI_E_STATE, "batch is full");
    s->row = free_rows_.back();
    free_rows_.pop_back();
    s->phase = BatchSlot::kStart;
    s->fp32 = s->o.precision == TBSCI_MIXED;
    if (s->guess) {  // a caller's start vector picks its own sector
        s->sector = 0;
        s->npass = 1;
    }
    s->pass = 0;
    s->t0 = std::chrono::steady_clock::now();
    memset(&s->info, 0, sizeof(s->info));
    s->info.lean = s->lean ? 1 : 0;
    act_.push_back(s);
}

std::vector<BatchSlot *> BatchEngine::take_done() {
    std::vector<BatchSlot *> d;
    d.swap(done_);
    return d;
}

std::vector<BatchSlot *> BatchEngine::drain() {
    std::vector<BatchSlot *> v, out;
    v.swap(act_);
    for (BatchSlot *s : v) {
        free_rows_.push_back(s->row);
        s->row = -1;
    }
    // report each solve once, by its primary slot (a held partner included)
    for (BatchSlot *s : v) {
        BatchSlot *p = s->primary ? s->primary : s;
        if (std::find(out.begin(), out.end(), p) == out.end()) out.push_back(p);
    }
    return out;
}

void BatchEngine::plan(BatchSlot &s, Stage &S) {
    auto &P = s.p;
    P = BatchSlot::Plan{};
    double *scal = scal_dev_ + (size_t)s.row * kScal;
    auto base = [&]() {
        VDesc d{};
        d.n = s.n;
        d.nb = s.nb;
        d.partial = s.partial;
        d.scal = scal;
        d.src2 = -1;
        return d;
    };
    auto dots = [&](int op, const std::vector<double *> &a, const double *in, int dst) {
        VDesc d = base();
        d.k = (int)a.size();
        for (int i = 0; i < d.k; ++i) d.a[i] = a[i];
        d.in = in;
        S.ops[op].push_back(d);
        VDesc r = base();
        r.k = d.k;
        r.dst = dst;
        S.ops[op + 1].push_back(r);
    };
    auto reduce = [&](int op, int k, int dst) {
        VDesc r = base();
        r.k = k;
        r.dst = dst;
        S.ops[op].push_back(r);
    };
    auto scale = [&](int op, double *o0, double *o1, int src, int src2, double thresh) {
        VDesc d = base();
        d.o0 = o0;
        d.o1 = o1;
        d.src = src;
        d.src2 = src2;
        d.thresh = thresh;
        S.ops[op].push_back(d);
    };
    auto diag_fields = [&](VDesc &d) {
        d.lb = s.c->sp[1].l;
        d.M = s.c->M;
        d.astr = s.c->sp[0].str;
        d.da = s.c->sp[0].dsame;
        d.db = s.c->sp[1].dsame;
        d.jb = s.c->sp[1].jocc;
        d.mask = s.c->dets ? s.c->dets->mask : nullptr;
        d.wpr = s.c->dets ? s.c->dets->wpr : 0;
    };
    // a TBSCI space: the sigma of a zero-extended vector, read on the space
    auto mask_out = [&](double *o) {
        if (!s.c->dets) return;
        VDesc m = base();
        diag_fields(m);
        m.o0 = o;
        S.ops[O_MASK].push_back(m);
    };
    auto take = [](std::vector<double *> &pool) {
        if (pool.empty()) throw Error(TBSCI_E_STATE, "batch slot vector pool exhausted");
        double *p = pool.back();
        pool.pop_back();
        return p;
    };

    if (s.phase == BatchSlot::kFinish) {
        // the pass's Ritz vector x: its signed copy to the output when it is
        // the lowest state so far, and a fresh FP64 sigma for x.x and x.Hx
        if (s.write_out) {
            VDesc m = base();
            m.in = s.X;
            S.ops[O_AMAX].push_back(m);
            VDesc g = base();
            g.in = s.X;
            g.dst = sSign;
            S.ops[O_AMAX_S].push_back(g);
            VDesc o = base();
            o.in = s.X;
            o.o0 = s.out;
            o.src = sSign;
            S.ops[O_OUT].push_back(o);
        }
        P.W0 = take(s.wfree);
        S.c64.push_back(s.c);
        S.i64.push_back(s.X);
        S.o64.push_back(P.W0);
        mask_out(P.W0);
        dots(O_COL_D, {s.X, P.W0}, s.X, sCol);
        return;
    }

    const double *sig_in = nullptr;
    double *sig_out = nullptr;
    if (s.phase == BatchSlot::kStart || s.phase == BatchSlot::kHandover) {
        if (s.phase == BatchSlot::kStart && s.diag && s.pass == 0) {
            VDesc dg = base();
            diag_fields(dg);
            dg.o0 = s.diag;
            S.ops[O_DIAG].push_back(dg);
        }
        const double *g = s.guess ? s.guess : s.pass_guess[std::min(s.pass, 1)];
        if (s.phase == BatchSlot::kStart && !g) {
            P.V0 = take(s.vfree);
            VDesc f = base();
            f.o0 = P.V0;
            S.ops[O_FILL].push_back(f);
            VDesc m = base();
            diag_fields(m);
            m.flip = s.sector;
            S.ops[O_DMIN].push_back(m);
            VDesc u = base();
            u.o0 = P.V0;
            u.dst = sArg;
            u.lb = s.c->sp[1].l;
            u.flip = s.sector;
            S.ops[O_AMIN].push_back(u);
        } else if (s.phase == BatchSlot::kStart) {
            P.V0 = take(s.vfree);
            VDesc cp = base();
            cp.o0 = P.V0;
            cp.in = g;
            S.ops[O_GCOPY].push_back(cp);
            dots(O_GN_D, {P.V0}, P.V0, sGN);
            scale(O_GN_S, P.V0, nullptr, sGN, -1, 0.0);
        } else {
            P.V0 = s.X;  // the Ritz vector of the FP32 phase
            s.X = nullptr;
        }
        P.W0 = take(s.wfree);
        P.sig32 = s.phase == BatchSlot::kStart && s.fp32;
        sig_in = P.V0;
        sig_out = P.W0;
        dots(O_COL_D, {P.V0}, P.W0, sCol);
    } else {
        // Rayleigh-Ritz on the k x k projected matrix
        const int k = s.k, nm = s.o.n_max;
        std::vector<double> Gk((size_t)k * k), w, Z;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) Gk[i * k + j] = 0.5 * (s.G[i * nm + j] + s.G[j * nm + i]);
        jacobi_eigh(k, Gk, w, Z);
        int lo = 0;
        for (int i = 1; i < k; ++i)
            if (w[i] < w[lo]) lo = i;
        s.theta_prev = s.theta;
        s.theta = w[lo];
        s.y.assign(k, 0.0);
        for (int i = 0; i < k; ++i) s.y[i] = Z[i * k + lo];
        std::vector<double> yp = s.yprev;
        yp.resize(k, 0.0);
        s.yprev = s.y;

        P.Xn = take(s.vfree);
        P.WXn = take(s.wfree);
        P.T = take(s.vfree);
        if (!(s.lean && k >= nm)) P.TW = take(s.wfree);  // else reused below
        P.sig32 = s.fp32;
        VDesc r = base();
        diag_fields(r);
        r.k = k;
        for (int i = 0; i < k; ++i) {
            r.a[i] = s.V[i];
            r.b[i] = s.W[i];
            r.c[i] = s.y[i];
        }
        r.theta = s.theta;
        r.floor_ = s.o.precond_floor;
        r.in = s.diag;
        r.o0 = P.Xn;
        r.o1 = P.WXn;
        r.o2 = P.T;
        S.ops[O_RITZ].push_back(r);
        reduce(O_RITZ_R, 1, sR2);
        if (s.sector != 0) {  // keep the solve in its sector C^T = sector C
            VDesc y = base();
            const int64_t l = s.c->sp[1].l, nt = (l + 31) / 32;
            y.nb = (int32_t)(nt * nt);
            y.lb = l;
            y.flip = s.sector;
            y.o0 = P.T;
            S.ops[O_SYM].push_back(y);
        }

        P.restart = k >= nm;
        if (P.restart && s.lean) {
            // plain collapse to the Ritz vector; the image of the correction
            // goes into a vector of the old W basis, which nothing reads after
            // the Ritz kernel (the sigma runs after it in stream order)
            dots(O_G0_D, {P.WXn}, P.Xn, sG);
            P.Vb = {P.Xn};
            P.Wb = {P.WXn};
            P.TW = s.W.back();
            P.tw_reused = true;
        } else if (P.restart) {
            // keep x = V y and the part of the previous Ritz vector
            // orthogonal to it, z = yp - (yp.y) y (when there is room)
            std::vector<double> z(k);
            double dz = 0.0, nz = 0.0;
            for (int i = 0; i < k; ++i) dz += yp[i] * s.y[i];
            for (int i = 0; i < k; ++i) {
                z[i] = yp[i] - dz * s.y[i];
                nz += z[i] * z[i];
            }
            nz = std::sqrt(nz);
            if (nz > 1e-8 && nm >= 3) {
                P.took_xp = true;
                P.XP = take(s.vfree);
                P.WXP = take(s.wfree);
                VDesc l = base();
                l.k = k;
                for (int i = 0; i < k; ++i) {
                    l.a[i] = s.V[i];
                    l.b[i] = s.W[i];
                    l.c[i] = z[i] / nz;
                }
                l.o0 = P.XP;
                l.o1 = P.WXP;
                S.ops[O_LC].push_back(l);
                // V z is a difference of nearly equal vectors near
                // convergence: re-orthogonalise against x twice, with the
                // same combination on its image
                for (int pass = 0; pass < 2; ++pass) {
                    const int op = pass == 0 ? O_RO1_D : O_RO2_D;
                    dots(op, {P.Xn}, P.XP, sRO);
                    VDesc sp = base();
                    sp.k = 1;
                    sp.a[0] = P.Xn;
                    sp.b[0] = P.WXn;
                    sp.o0 = P.XP;
                    sp.o1 = P.WXP;
                    sp.src = sRO;
                    S.ops[op + 2].push_back(sp);
                }
                dots(O_N2_D, {P.XP}, P.XP, sN2);
                scale(O_N2_S, P.XP, P.WXP, sN2, -1, 1e-8);
                dots(O_G0_D, {P.WXn, P.WXP}, P.Xn, sG);
                dots(O_G1_D, {P.WXn, P.WXP}, P.XP, sG + 2);
                P.Vb = {P.Xn, P.XP};
                P.Wb = {P.WXn, P.WXP};
            } else {
                dots(O_G0_D, {P.WXn}, P.Xn, sG);
                P.Vb = {P.Xn};
                P.Wb = {P.WXn};
            }
        } else {
            P.Vb = s.V;
            P.Wb = s.W;
        }
        // two Gram-Schmidt passes against the basis t joins, then t is
        // normalised; a t left with at most 1e-10 of its norm is dropped
        const int kb = (int)P.Vb.size();
        std::vector<double *> with_t = P.Vb;
        with_t.push_back(P.T);
        dots(O_D1, with_t, P.T, sD1);  // coefficients, and |t|^2 at sD1 + kb
        VDesc sd = base();
        sd.k = kb;
        for (int i = 0; i < kb; ++i) sd.a[i] = P.Vb[i];
        sd.o0 = P.T;
        sd.src = sD1;
        S.ops[O_S1D2].push_back(sd);
        reduce(O_S1D2_R, kb, sD2);
        VDesc sn = sd;
        sn.src = sD2;
        S.ops[O_S2N].push_back(sn);
        reduce(O_S2N_R, 1, sTn2);
        scale(O_TSCALE, P.T, nullptr, sTn2, sD1 + kb, 1e-10);
        sig_in = P.T;
        sig_out = P.TW;
        dots(O_COL_D, with_t, P.TW, sCol);
    }
    mask_out(sig_out);
    if (P.sig32) {
        VDesc a = base();
        a.in = sig_in;
        a.f = s.f32a;
        S.ops[O_CVT32].push_back(a);
        S.c32.push_back(s.c);
        S.i32.push_back(s.f32a);
        S.o32.push_back(s.f32b);
        VDesc b = base();
        b.f = s.f32b;
        b.o0 = sig_out;
        S.ops[O_CVT64].push_back(b);
    } else {
        S.c64.push_back(s.c);
        S.i64.push_back(sig_in);
        S.o64.push_back(sig_out);
    }
}

bool BatchEngine::tick() {
    if (act_.empty()) return false;
    TB_HIP(hipSetDevice(device_));
    ar_.reset();
    Stage S;
    for (BatchSlot *s : act_) plan(*s, S);
    max_group = std::max(max_group, (int)act_.size());

    // stage every table of the round, one transfer
    const VDesc *dev[O_N] = {};
    int64_t blocks[O_N] = {};
    int kmax[O_N] = {};
    for (int op = 0; op < O_N; ++op) {
        auto &v = S.ops[op];
        if (v.empty()) continue;
        const Kind kd = kind_of(op);
        if (kd == K_RED) {
            for (auto &d : v) kmax[op] = std::max(kmax[op], (int)d.k);
            blocks[op] = (int64_t)v.size() * kmax[op];
        } else if (kd == K_AMIN || kd == K_ASIGN) {
            blocks[op] = (int64_t)v.size();
        } else {
            int64_t b = 0;
            for (auto &d : v) {
                d.blk0 = b;
                b += d.nb;
            }
            blocks[op] = b;
        }
        dev[op] = ar_.stage(v.data(), v.size());
    }
    ar_.flush(st_);

    auto launch = [&](int op) {
        if (S.ops[op].empty()) return;
        const unsigned g = (unsigned)blocks[op];
        const int nd = (int)S.ops[op].size();
        const VDesc *d = dev[op];
        switch (kind_of(op)) {
            case K_DIAG: gv_diag<<<g, kB, 0, st_>>>(d, nd); break;
            case K_FILL: gv_fill<<<g, kB, 0, st_>>>(d, nd); break;
            case K_COPY: gv_copy<<<g, kB, 0, st_>>>(d, nd); break;
            case K_DMIN: gv_diag_min<<<g, kB, 0, st_>>>(d, nd); break;
            case K_AMIN: gv_argmin_unit<<<g, kB, 0, st_>>>(d); break;
            case K_AMAX: gv_absmax<<<g, kB, 0, st_>>>(d, nd); break;
            case K_ASIGN: gv_absmax_sign<<<g, kB, 0, st_>>>(d); break;
            case K_SCOPY: gv_signed_copy<<<g, kB, 0, st_>>>(d, nd); break;
            case K_RITZ: gv_ritz<<<g, kB, 0, st_>>>(d, nd); break;
            case K_RED: gv_reduce<<<g, kB, 0, st_>>>(d, kmax[op]); break;
            case K_SYM: gv_flip_sym<<<g, kB, 0, st_>>>(d, nd); break;
            case K_LC: gv_lincomb2<<<g, kB, 0, st_>>>(d, nd); break;
            case K_DOT: gv_dots<<<g, kB, 0, st_>>>(d, nd); break;
            case K_SUB: gv_subproj<<<g, kB, 0, st_>>>(d, nd); break;
            case K_SUBDOT: gv_subdots<<<g, kB, 0, st_>>>(d, nd); break;
            case K_SUBNORM: gv_subnorm<<<g, kB, 0, st_>>>(d, nd); break;
            case K_SCALE: gv_scale<<<g, kB, 0, st_>>>(d, nd); break;
            case K_F32: gv_to_f32<<<g, kB, 0, st_>>>(d, nd); break;
            case K_F64: gv_to_f64<<<g, kB, 0, st_>>>(d, nd); break;
            case K_MASK: gv_mask<<<g, kB, 0, st_>>>(d, nd); break;
            case K_NONE: break;
        }
        TB_HIP(hipGetLastError());
    };
    for (int op = 0; op < O_SIGMA; ++op) launch(op);
    const bool sig = !S.c64.empty() || !S.c32.empty();
    TB_HIP(hipEventRecord(ev_[0], st_));
    if (!S.c64.empty())
        launch_sigma_group(S.c64.data(), S.i64.data(), S.o64.data(), (int)S.c64.size(),
                           TBSCI_FP64, ar_, st_);
    if (!S.c32.empty())
        launch_sigma_group(S.c32.data(), S.i32.data(), S.o32.data(), (int)S.c32.size(),
                           TBSCI_FP32, ar_, st_);
    launch(O_CVT64);
    TB_HIP(hipEventRecord(ev_[1], st_));
    for (int op = O_CVT64 + 1; op < O_N; ++op) launch(op);

    int rows = 0;
    for (BatchSlot *s : act_) rows = std::max(rows, s->row + 1);
    TB_HIP(hipMemcpyAsync(scal_host_, scal_dev_, sizeof(double) * kScal * rows,
                          hipMemcpyDeviceToHost, st_));
    TB_HIP(hipStreamSynchronize(st_));
    float ms = 0.f;
    if (sig) TB_HIP(hipEventElapsedTime(&ms, ev_[0], ev_[1]));
    ++ticks;

    std::vector<BatchSlot *> still;
    for (BatchSlot *s : act_) {
        commit(*s, scal_host_ + (size_t)s->row * kScal, ms * 1e-3);
        if (s->phase == BatchSlot::kDone) {
            free_rows_.push_back(s->row);
            s->row = -1;
            BatchSlot *partner = s->twin ? s->twin : s->primary;
            if (!partner) {
                done_.push_back(s);
            } else if (partner->held) {  // both sectors done: one result
                BatchSlot *p = s->primary ? s->primary : s;
                merge_twins(*p);
                done_.push_back(p);
            } else {
                s->held = true;
            }
        } else {
            still.push_back(s);
        }
    }
    act_.swap(still);
    return true;
}

// Result of a split two-sector solve from its two slots: the lower state,
// the other sector's energy, iterations of both, wall time of the longer.
void BatchEngine::merge_twins(BatchSlot &p) {
    BatchSlot &q = *p.twin;
    const bool q_low = q.info.energy < p.info.energy;
    const tbsci_davidson_info a = p.info, b = q.info;
    const tbsci_davidson_info &lo = q_low ? b : a, &hi = q_low ? a : b;
    p.info = lo;
    p.info.energy_other = hi.energy;
    p.info.iters = a.iters + b.iters;
    p.info.iters_fp32 = a.iters_fp32 + b.iters_fp32;
    p.info.iters_fp64 = a.iters_fp64 + b.iters_fp64;
    p.info.converged = (a.converged && b.converged) ? 1 : 0;
    p.info.t_total_s = std::max(a.t_total_s, b.t_total_s);
    p.info.t_sigma_s = std::max(a.t_sigma_s, b.t_sigma_s);
    int st = p.status;
    if (q.status != TBSCI_OK && q.status != TBSCI_E_NOTCONV) st = q.status;
    else if (st == TBSCI_OK && q.status != TBSCI_OK) st = q.status;
    p.status = st;
    if (st == TBSCI_E_INVAL) p.msg = q.status == TBSCI_E_INVAL ? q.msg : p.msg;
    p.held = q.held = false;
}

// A pass has ended with Ritz vector x: one more round (kFinish) checks its
// energy with a fresh FP64 sigma build and writes the output vector when x
// is the lowest state so far.  x == nullptr: the solve ended with an error.
void BatchEngine::finish(BatchSlot &s, double *x) {
    if (s.fp32) s.pass_conv = false;  // never certified by an FP64 sigma
    if (!x) {
        complete(s);
        return;
    }
    s.X = x;
    s.write_out = s.out && (!s.best.valid || s.theta < s.best.e);
    s.phase = BatchSlot::kFinish;
}

// the solve's result from its passes (the lowest state found)
void BatchEngine::complete(BatchSlot &s) {
    if (s.best.valid) {
        s.info.energy = s.best.e;
        s.info.resid_norm = s.best.rn;
        s.info.energy_fp64_check = s.best.echk;
        s.info.sector = s.best.sector;
    } else {
        s.info.energy = s.theta;
        s.info.resid_norm = s.rn;
        s.info.energy_fp64_check = std::nan("");
        s.info.sector = s.sector;
    }
    s.info.energy_other = s.have_other ? s.e_other : std::nan("");
    s.info.converged = (s.best.valid && s.all_conv) ? 1 : 0;
    if (s.status == TBSCI_PENDING) s.status = s.info.converged ? TBSCI_OK : TBSCI_E_NOTCONV;
    s.phase = BatchSlot::kDone;
    s.info.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - s.t0).count();
}

void BatchEngine::commit(BatchSlot &s, const double *r, double t_sig) {
    auto &P = s.p;
    const int nm = s.o.n_max;
    if (s.phase == BatchSlot::kFinish) {
        s.info.iters++;
        s.info.iters_fp64++;
        s.info.t_sigma_s += t_sig;
        BatchSlot::PassResult cur;
        cur.valid = true;
        cur.e = s.theta;
        cur.rn = s.rn;
        cur.echk = r[sCol] > 0.0 ? r[sCol + 1] / r[sCol] : std::nan("");
        cur.sector = s.sector;
        s.all_conv = s.all_conv && s.pass_conv;
        if (!s.best.valid || cur.e < s.best.e) {
            if (s.best.valid) {
                s.e_other = s.best.e;
                s.have_other = true;
            }
            s.best = cur;
        } else {
            s.e_other = cur.e;
            s.have_other = true;
        }
        s.vfree.push_back(s.X);
        s.X = nullptr;
        s.wfree.push_back(P.W0);
        if (s.pass + 1 < s.npass) {  // the antisymmetric sector, from its own start
            s.pass++;
            s.sector = -1;
            s.phase = BatchSlot::kStart;
            s.fp32 = s.o.precision == TBSCI_MIXED;
            s.k = 0;
            s.V.clear();
            s.W.clear();
            s.yprev.clear();
            s.theta = s.theta_prev = 0.0;
            s.rn = s.best_rn = 1e300;
            s.since_best = 0;
            s.pass_conv = false;
            return;
        }
        complete(s);
        return;
    }
    s.info.iters++;
    if (P.sig32)
        s.info.iters_fp32++;
    else
        s.info.iters_fp64++;
    s.info.t_sigma_s += t_sig;
    auto release_v = [&](double *p) {
        if (p) s.vfree.push_back(p);
    };
    auto release_w = [&](double *p) {
        if (p) s.wfree.push_back(p);
    };

    if (s.phase == BatchSlot::kStart || s.phase == BatchSlot::kHandover) {
        const bool had_guess = s.guess || s.pass_guess[std::min(s.pass, 1)];
        if (s.phase == BatchSlot::kStart && had_guess && !(r[sGN] > 0.0)) {
            release_v(P.V0);
            release_w(P.W0);
            s.status = TBSCI_E_INVAL;
            s.msg = "guess vector is zero";
            finish(s, nullptr);
            return;
        }
        if (s.phase == BatchSlot::kHandover) s.fp32 = false;
        s.V = {P.V0};
        s.W = {P.W0};
        std::fill(s.G.begin(), s.G.end(), 0.0);
        s.G[0] = r[sCol];
        s.k = 1;
        s.theta = r[sCol];
        s.yprev.clear();
        s.phase = BatchSlot::kIter;
        return;
    }

    s.rn = std::sqrt(std::max(r[sR2], 0.0));
    const int kb = (int)P.Vb.size();
    const double t0n = std::sqrt(std::max(r[sD1 + kb], 0.0));
    const double tn = std::sqrt(std::max(r[sTn2], 0.0));
    const bool dropped = !(tn > 1e-10 * t0n);
    if (trace)
        fprintf(stderr, "tbsci davidson: sigma %d k %d %s theta %.15f resid %.3e\n", s.info.iters,
                s.k, s.fp32 ? "fp32" : "fp64", s.theta, s.rn);

    // everything of this round except the Ritz vector goes back to the pools
    auto drop_all_but_x = [&]() {
        for (double *p : s.V) release_v(p);
        for (double *p : s.W) release_w(p);
        s.V.clear();
        s.W.clear();
        release_w(P.WXn);
        release_v(P.T);
        if (!P.tw_reused) release_w(P.TW);  // else it was one of s.W
        release_v(P.XP);
        release_w(P.WXP);
    };
    bool handover = false;
    if (s.fp32) {
        // The FP32 phase ends at fp32_switch_resid, or when the residual
        // has stopped improving for 30 iterations within 2x of the FP32
        // rounding floor of the sigma build (taken as 2e-6 |theta|), or at
        // half the iteration budget, or when no new direction is left.  A
        // plateau above that is slow convergence, which FP64 would not cure
        // (FP64 solves of the same problems show plateaus of 40 iterations).
        if (s.rn < 0.98 * s.best_rn) {
            s.best_rn = s.rn;
            s.since_best = 0;
        } else {
            ++s.since_best;
        }
        const bool at_floor = s.rn < 2.0 * 2e-6 * std::fabs(s.theta);
        handover = s.rn <= s.o.fp32_switch_resid || (s.since_best >= 30 && at_floor) ||
                   s.info.iters >= s.o.max_iter / 2 || dropped;
    } else if (s.rn <= s.o.tol_resid &&
               (s.o.tol_energy <= 0.0 || std::fabs(s.theta - s.theta_prev) <= s.o.tol_energy)) {
        s.pass_conv = true;
        drop_all_but_x();
        finish(s, P.Xn);
        return;
    }
    if (!handover && (s.info.iters >= s.o.max_iter || (!s.fp32 && dropped))) {
        drop_all_but_x();
        finish(s, P.Xn);  // not converged (iteration cap or stagnation)
        return;
    }
    if (handover) {
        drop_all_but_x();
        s.X = P.Xn;
        s.phase = BatchSlot::kHandover;
        return;
    }
    // the restart (if any) becomes the basis; positions of its vectors in
    // the column of dots
    std::vector<int> pos;
    if (P.restart) {
        for (double *p : s.V) release_v(p);
        for (double *p : s.W)
            if (!(P.tw_reused && p == P.TW)) release_w(p);
        const bool two = P.took_xp && std::sqrt(std::max(r[sN2], 0.0)) > 1e-8;
        std::fill(s.G.begin(), s.G.end(), 0.0);
        if (two) {
            s.V = {P.Xn, P.XP};
            s.W = {P.WXn, P.WXP};
            s.G[0] = r[sG];
            s.G[1] = r[sG + 1];
            s.G[nm] = r[sG + 2];
            s.G[nm + 1] = r[sG + 3];
            s.yprev = {1.0, 0.0};
            pos = {0, 1};
        } else {
            release_v(P.XP);
            release_w(P.WXP);
            s.V = {P.Xn};
            s.W = {P.WXn};
            s.G[0] = r[sG];
            s.yprev = {1.0};
            pos = {0};
        }
        s.k = (int)s.V.size();
    } else {
        release_v(P.Xn);
        release_w(P.WXn);
        for (int i = 0; i < s.k; ++i) pos.push_back(i);
    }
    s.V.push_back(P.T);
    s.W.push_back(P.TW);
    pos.push_back(kb);
    const int kk = s.k;  // index of the new vector
    for (int i = 0; i <= kk; ++i) s.G[i * nm + kk] = s.G[kk * nm + i] = r[sCol + pos[i]];
    s.k = kk + 1;
}

namespace {

// G[ma[i]][mb[j]] = X[i][j] for the ka x kb subspace vector X (G zeroed)
__global__ __launch_bounds__(kB) void k_embed(int64_t ka, int64_t kb, int64_t lb,
                                              const int32_t *__restrict__ ma,
                                              const int32_t *__restrict__ mb,
                                              const double *__restrict__ X,
                                              double *__restrict__ G) {
    const int64_t n = ka * kb;
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kB) {
        const int64_t i = t / kb, j = t - i * kb;
        G[(int64_t)ma[i] * lb + mb[j]] = X[t];
    }
}

__global__ __launch_bounds__(kB) void k_zero64(int64_t n, double *__restrict__ o) {
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kB)
        o[t] = 0.0;
}

template <typename T>
std::vector<T> to_host(const T *d, size_t n) {
    std::vector<T> h(n);
    TB_HIP(hipMemcpy(h.data(), d, sizeof(T) * n, hipMemcpyDeviceToHost));
    return h;
}

// Start vectors of the passes of a solve from a subspace (a P-space
// start): the k strings of each spin with the smallest same-spin diagonal
// (the same strings for both spins of identical lists), that space solved
// in FP64 per sector, each solution extended by zeros.  Returns the device
// vectors (one per pass) and adds the time spent to *secs.
std::vector<double *> subspace_guesses(Ctx &c, const tbsci_davidson_opts &o,
                                       const std::vector<int> &sectors, hipStream_t st,
                                       double *secs) {
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<double *> out;
    Ctx *sub = nullptr;
    int32_t *dmap = nullptr;
    double *X = nullptr;
    try {
        const int M = c.M;
        const int64_t la = c.sp[0].l, lb = c.sp[1].l;
        auto pick = [&](const Spin &sp) {
            int64_t k = o.guess_strings > 0 ? (int64_t)o.guess_strings
                                            : std::max<int64_t>((sp.l + 4) / 5, 50);
            k = std::min(k, sp.l);
            const std::vector<double> d = to_host(sp.dsame, (size_t)sp.l);
            std::vector<int32_t> idx((size_t)sp.l);
            for (int64_t i = 0; i < sp.l; ++i) idx[(size_t)i] = (int32_t)i;
            std::stable_sort(idx.begin(), idx.end(),
                             [&](int32_t a, int32_t b) { return d[(size_t)a] < d[(size_t)b]; });
            idx.resize((size_t)k);
            std::sort(idx.begin(), idx.end());  // keep the caller's order
            return idx;
        };
        const std::vector<int32_t> ia = pick(c.sp[0]);
        const std::vector<int32_t> ib = c.flip ? ia : pick(c.sp[1]);
        const std::vector<uint64_t> sa = to_host(c.sp[0].str, (size_t)la);
        const std::vector<uint64_t> sb = to_host(c.sp[1].str, (size_t)lb);
        std::vector<uint64_t> ua, ub;
        for (int32_t i : ia) ua.push_back(sa[(size_t)i]);
        for (int32_t i : ib) ub.push_back(sb[(size_t)i]);
        const std::vector<double> h = to_host(c.h, (size_t)M * M);
        const std::vector<double> eri = to_host(c.eri, (size_t)M * M * M * M);
        sub = create_ctx(M, c.sp[0].n, c.sp[1].n, h.data(), eri.data(), ua.data(),
                         (int64_t)ua.size(), ub.data(), (int64_t)ub.size(), c.device);
        const int64_t ka = (int64_t)ua.size(), kb = (int64_t)ub.size();
        TB_HIP(hipMalloc((void **)&dmap, sizeof(int32_t) * (ka + kb)));
        TB_HIP(hipMemcpy(dmap, ia.data(), sizeof(int32_t) * ka, hipMemcpyHostToDevice));
        TB_HIP(hipMemcpy(dmap + ka, ib.data(), sizeof(int32_t) * kb, hipMemcpyHostToDevice));
        TB_HIP(hipMalloc((void **)&X, sizeof(double) * ka * kb));
        for (int sec : sectors) {
            tbsci_davidson_opts os = o;
            os.precision = TBSCI_FP64;
            os.guess_kind = TBSCI_GUESS_DIAG;
            os.storage = TBSCI_STORE_FULL;
            os.sector = sec;
            os.tol_resid = std::max(o.tol_resid, 1e-3);
            os.tol_energy = 0.0;
            tbsci_davidson_info si{};
            (void)solve_one(*sub, os, nullptr, X, si, st);
            double *G = nullptr;
            TB_HIP(hipMalloc((void **)&G, sizeof(double) * la * lb));
            out.push_back(G);
            const int64_t n = la * lb, m = ka * kb;
            k_zero64<<<(unsigned)std::min<int64_t>((n + kB - 1) / kB, 16384), kB, 0, st>>>(n, G);
            k_embed<<<(unsigned)std::min<int64_t>((m + kB - 1) / kB, 16384), kB, 0, st>>>(
                ka, kb, lb, dmap, dmap + ka, X, G);
            TB_HIP(hipGetLastError());
        }
        TB_HIP(hipStreamSynchronize(st));
    } catch (...) {
        (void)hipStreamSynchronize(st);
        for (double *g : out) (void)hipFree(g);
        if (X) (void)hipFree(X);
        if (dmap) (void)hipFree(dmap);
        destroy_ctx(sub);
        throw;
    }
    (void)hipFree(X);
    (void)hipFree(dmap);
    destroy_ctx(sub);
    *secs += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return out;
}

}  // namespace

int solve_one(Ctx &c, const tbsci_davidson_opts &o, const double *guess, double *out,
              tbsci_davidson_info &info, hipStream_t st, const std::atomic<bool> *abort) {
    reserve_sigma_workspace(c);
    // a subspace start: one start vector per sector the solve will run
    std::vector<double *> pg;
    double sub_s = 0.0;
    if (o.guess_kind == TBSCI_GUESS_SUBSPACE && !guess) {
        if (c.dets) throw Error(TBSCI_E_INVAL, "subspace starts need the whole TPB space");
        std::vector<int> secs;
        if (!c.flip) {
            secs = {0};
        } else if (o.sector != 0) {
            secs = {o.sector};
        } else {
            secs = {1};
            if (c.sp[0].l >= 2) secs.push_back(-1);
        }
        if (c.flip && o.sector == -1 && c.sp[0].l < 2)
            throw Error(TBSCI_E_INVAL, "the antisymmetric sector of this space is empty");
        pg = subspace_guesses(c, o, secs, st, &sub_s);
    }
    struct FreeG {
        std::vector<double *> &v;
        ~FreeG() {
            for (double *g : v) (void)hipFree(g);
        }
    } free_g{pg};
    BatchSlot *s = BatchEngine::make_slot(&c, o, guess != nullptr);
    s->guess = guess;
    s->out = out;
    for (size_t i = 0; i < pg.size() && i < 2; ++i) s->pass_guess[i] = pg[i];
    int rc = TBSCI_OK;
    try {
        BatchEngine eng(c.device, st);
        const char *tr = getenv("TBSCI_DAVIDSON_TRACE");  // per-iteration trace on stderr
        eng.trace = tr && tr[0] && tr[0] != '0';
        eng.add(s);
        bool aborted = false;
        while (eng.tick())
            if (abort && abort->load()) {
                aborted = true;
                break;
            }
        info = s->info;
        info.t_total_s += sub_s;
        if (aborted) {
            eng.drain();
            info.energy = s->theta;
            info.resid_norm = s->rn;
            info.converged = 0;
            rc = TBSCI_E_STATE;
        } else {
            rc = s->status;
            if (rc == TBSCI_E_INVAL) throw Error(rc, s->msg);
        }
    } catch (...) {
        (void)hipStreamSynchronize(st);
        BatchEngine::free_slot(s);
        throw;
    }
    BatchEngine::free_slot(s);
    return rc;
}

}  // namespace tbsci

using namespace tbsci;

extern "C" {

int tbsci_davidson(tbsci_ctx *ctx, const tbsci_davidson_opts *opts, const double *guess_dev,
                   double *C_out_dev, tbsci_davidson_info *info, void *stream) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        Ctx *c = ctx_of(ctx);
        if (!info) throw Error(TBSCI_E_INVAL, "info is NULL");
        tbsci_davidson_opts o;
        tbsci_davidson_default_opts(&o);
        if (opts) o = *opts;
        check_opts(o);
        if ((o.guess_kind == TBSCI_GUESS_USER) != (guess_dev != nullptr))
            throw Error(TBSCI_E_INVAL, "guess_dev must be given exactly when guess_kind is "
                                       "TBSCI_GUESS_USER");
        if (guess_dev) check_dev(guess_dev, c->device, "guess");
        if (C_out_dev) check_dev(C_out_dev, c->device, "C_out");
        hipStream_t st = (hipStream_t)stream;
        // a TBSCI space: the solver works on zero-extended vectors; the
        // guess and the output are compact at the boundary
        const double *g = guess_dev;
        double *out = C_out_dev, *gd = nullptr, *od = nullptr;
        struct Free {
            double **p[2];
            ~Free() {
                for (double **q : p)
                    if (*q) (void)hipFree(*q);
            }
        } fr{{&gd, &od}};
        if (c->dets) {
            const size_t bytes = sizeof(double) * (size_t)(c->sp[0].l * c->sp[1].l);
            if (guess_dev) {
                TB_HIP(hipMalloc((void **)&gd, bytes));
                dets_expand(*c, guess_dev, gd, 8, st);
                g = gd;
            }
            if (C_out_dev) {
                TB_HIP(hipMalloc((void **)&od, bytes));
                out = od;
            }
        }
        tbsci_davidson_info tmp;
        const int rc = solve_one(*c, o, g, out, tmp, st);
        if (od) {
            dets_gather(*c, od, C_out_dev, 8, st);
            TB_HIP(hipStreamSynchronize(st));
        }
        *info = tmp;
        if (rc == TBSCI_E_NOTCONV) set_error(rc, "Davidson did not reach the tolerance");
        return rc;
    });
}

int tbsci_sigma_batch(tbsci_ctx *const *ctxs, int n, const void *const *C_dev,
                      void *const *sigma_dev, int precision, void *stream) {
    return guarded([&]() -> int {
        if (n < 0 || n > kBatchMaxSlots) throw Error(TBSCI_E_INVAL, "n must be in [0, 64]");
        if (n == 0) return TBSCI_OK;
        if (!ctxs || !C_dev || !sigma_dev) throw Error(TBSCI_E_INVAL, "NULL array");
        if (precision != TBSCI_FP64 && precision != TBSCI_FP32)
            throw Error(TBSCI_E_INVAL, "precision must be TBSCI_FP64 or TBSCI_FP32");
        std::vector<Ctx *> cs(n);
        for (int i = 0; i < n; ++i) {
            check_ctx(ctxs[i]);
            cs[i] = ctx_of(ctxs[i]);
            if (cs[i]->device != cs[0]->device)
                throw Error(TBSCI_E_INVAL, "contexts are on different devices");
            if (cs[i]->dets)
                throw Error(TBSCI_E_INVAL, "tbsci_sigma_batch takes whole TPB spaces only");
            check_dev(C_dev[i], cs[i]->device, "C");
            check_dev(sigma_dev[i], cs[i]->device, "sigma");
            if (C_dev[i] == sigma_dev[i]) throw Error(TBSCI_E_INVAL, "C and sigma must not alias");
            for (int j = 0; j < i; ++j)
                if (cs[j] == cs[i]) throw Error(TBSCI_E_INVAL, "a context appears twice");
        }
        TB_HIP(hipSetDevice(cs[0]->device));
        for (Ctx *c : cs) reserve_sigma_workspace(*c);
        TableArena ar(64u << 10);
        hipStream_t st = (hipStream_t)stream;
        launch_sigma_group(cs.data(), C_dev, sigma_dev, n, precision, ar, st);
        TB_HIP(hipStreamSynchronize(st));
        return TBSCI_OK;
    });
}

int tbsci_davidson_batch(tbsci_ctx *const *ctxs, int n, const tbsci_davidson_opts *opts,
                         tbsci_davidson_info *infos, int *status, void *stream) {
    return guarded([&]() -> int {
        if (n < 0 || n > kBatchMaxSlots) throw Error(TBSCI_E_INVAL, "n must be in [0, 64]");
        if (n == 0) return TBSCI_OK;
        if (!ctxs || !infos || !status) throw Error(TBSCI_E_INVAL, "NULL array");
        std::vector<Ctx *> cs(n);
        std::vector<tbsci_davidson_opts> os(n);
        for (int i = 0; i < n; ++i) {
            check_ctx(ctxs[i]);
            cs[i] = ctx_of(ctxs[i]);
            if (cs[i]->device != cs[0]->device)
                throw Error(TBSCI_E_INVAL, "contexts are on different devices");
            for (int j = 0; j < i; ++j)
                if (cs[j] == cs[i]) throw Error(TBSCI_E_INVAL, "a context appears twice");
            if (opts)
                os[i] = opts[i];
            else
                tbsci_davidson_default_opts(&os[i]);
            check_opts(os[i]);
            if (os[i].guess_kind != TBSCI_GUESS_DIAG)
                throw Error(TBSCI_E_INVAL, "batched solves take no start vector");
        }
        TB_HIP(hipSetDevice(cs[0]->device));
        hipStream_t st = (hipStream_t)stream;
        std::vector<BatchSlot *> slots;
        try {
            BatchEngine eng(cs[0]->device, st);
            const char *tr = getenv("TBSCI_DAVIDSON_TRACE");
            eng.trace = tr && tr[0] && tr[0] != '0';
            for (int i = 0; i < n; ++i) {
                reserve_sigma_workspace(*cs[i]);
                slots.push_back(BatchEngine::make_slot(cs[i], os[i], false, true));
                slots.back()->user = (void *)(intptr_t)i;
            }
            // two-sector problems add two slots; the rest wait for room
            size_t next = 0, running = 0;
            std::vector<BatchSlot *> fin;
            for (;;) {
                while (next < slots.size() &&
                       running + BatchEngine::slots_of(slots[next]) <= (size_t)kBatchMaxSlots) {
                    running += BatchEngine::slots_of(slots[next]);
                    eng.add(slots[next++]);
                }
                if (!eng.tick()) break;
                for (BatchSlot *s : eng.take_done()) {
                    running -= BatchEngine::slots_of(s);
                    fin.push_back(s);
                }
            }
            for (BatchSlot *s : fin) {
                const int i = (int)(intptr_t)s->user;
                infos[i] = s->info;
                status[i] = s->status;
            }
        } catch (...) {
            (void)hipStreamSynchronize(st);
            for (BatchSlot *s : slots) BatchEngine::free_slot(s);
            throw;
        }
        for (BatchSlot *s : slots) BatchEngine::free_slot(s);
        return TBSCI_OK;
    });
}

}  // extern "C"
