// String weights, weight-threshold selection and coefficient histograms
// (paper Sec. III.B: the weight of an alpha or beta string is the sum of the
// squared coefficients of the normalised CI vector over the determinants
// that contain it; strings are ranked by weight and kept when the weight
// exceeds delta times that of the Hartree-Fock string; the histograms of the
// coefficient magnitudes characterise the wavefunction).
//
// Reductions run in a fixed order (one block per alpha row; fixed row
// chunks for the beta weights, summed chunk by chunk), so weights are
// reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "tbsci_internal.hpp"

namespace tbsci {
namespace {

constexpr int kB = 256;
constexpr int64_t kRowChunk = 256;  // alpha rows per partial beta-weight sum

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// wa[w] = sum_u C[w][u]^2, one block per row
__global__ __launch_bounds__(kB) void k_row_weights(int64_t lb, const double *__restrict__ C,
                                                    double *__restrict__ wa) {
    __shared__ double red[kB / 64];
    const int64_t w = blockIdx.x;
    double s = 0.0;
    for (int64_t u = threadIdx.x; u < lb; u += kB) {
        const double c = C[w * lb + u];
        s += c * c;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kB / 64; ++i) t += red[i];
        wa[w] = t;
    }
}

// part[ch][u] = sum over rows of chunk ch of C[w][u]^2
__global__ __launch_bounds__(kB) void k_col_partial(int64_t la, int64_t lb,
                                                    const double *__restrict__ C,
                                                    double *__restrict__ part) {
    const int64_t u = (int64_t)blockIdx.x * kB + threadIdx.x;
    const int64_t ch = blockIdx.y;
    if (u >= lb) return;
    const int64_t w1 = std::min<int64_t>(la, (ch + 1) * kRowChunk);
    double s = 0.0;
    for (int64_t w = ch * kRowChunk; w < w1; ++w) {
        const double c = C[w * lb + u];
        s += c * c;
    }
    part[ch * lb + u] = s;
}

__global__ __launch_bounds__(kB) void k_col_reduce(int64_t lb, int64_t nch,
                                                   const double *__restrict__ part,
                                                   double *__restrict__ wb) {
    const int64_t u = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (u >= lb) return;
    double s = 0.0;
    for (int64_t ch = 0; ch < nch; ++ch) s += part[ch * lb + u];
    wb[u] = s;
}

// histogram of log10 |c| over [lo, hi) in nb bins; entries below lo (zeros
// included) go to bin 0 when clamp, entries at or above hi to bin nb-1
__global__ __launch_bounds__(kB) void k_hist(int64_t n, const double *__restrict__ c, double lo,
                                             double hi, int nb,
                                             unsigned long long *__restrict__ counts) {
    extern __shared__ unsigned int h[];
    for (int i = threadIdx.x; i < nb; i += kB) h[i] = 0;
    __syncthreads();
    const double scale = nb / (hi - lo);
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kB) {
        const double a = fabs(c[i]);
        int b = 0;
        if (a > 0.0) {
            const double x = (log10(a) - lo) * scale;
            b = x < 0.0 ? 0 : (x >= nb ? nb - 1 : (int)x);
        }
        atomicAdd(&h[b], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += kB)
        if (h[i]) atomicAdd(&counts[i], (unsigned long long)h[i]);
}

// flags[i] = w[i] > thresh
__global__ __launch_bounds__(kB) void k_over(int64_t l, const double *__restrict__ w, double thresh,
                                             int32_t *__restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < l) flags[i] = w[i] > thresh ? 1 : 0;
}

// a dense [l_alpha][l_beta] FP64 copy of a context vector: the vector itself
// for the TPB space, the zero-extended copy (context work) for a TBSCI space
const double *dense_of(Ctx &c, const double *C, hipStream_t st) {
    if (!c.dets) return C;
    double *X = dets_work(c);
    dets_expand(c, C, X, 8, st);
    return X;
}

}  // namespace
}  // namespace tbsci

using namespace tbsci;

extern "C" {

int tbsci_string_weights(tbsci_ctx *ctx, const double *C_dev, double *w_alpha_dev,
                         double *w_beta_dev, void *stream) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        Ctx *c = ctx_of(ctx);
        check_dev(C_dev, c->device, "C");
        check_dev(w_alpha_dev, c->device, "w_alpha");
        check_dev(w_beta_dev, c->device, "w_beta");
        hipStream_t st = (hipStream_t)stream;
        const int64_t la = c->sp[0].l, lb = c->sp[1].l;
        const double *X = dense_of(*c, C_dev, st);
        k_row_weights<<<(unsigned)la, kB, 0, st>>>(lb, X, w_alpha_dev);
        const int64_t nch = (la + kRowChunk - 1) / kRowChunk;
        double *part = nullptr;
        TB_HIP(hipMalloc((void **)&part, sizeof(double) * (size_t)(nch * lb)));
        const unsigned gx = (unsigned)((lb + kB - 1) / kB);
        k_col_partial<<<dim3(gx, (unsigned)nch), kB, 0, st>>>(la, lb, X, part);
        k_col_reduce<<<gx, kB, 0, st>>>(lb, nch, part, w_beta_dev);
        TB_HIP(hipGetLastError());
        TB_HIP(hipStreamSynchronize(st));
        TB_HIP(hipFree(part));
        return TBSCI_OK;
    });
}

int tbsci_coef_histogram(tbsci_ctx *ctx, const double *C_dev, double log10_lo, double log10_hi,
                         int nbins, int64_t *counts_host, void *stream) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        Ctx *c = ctx_of(ctx);
        check_dev(C_dev, c->device, "C");
        if (!counts_host) throw Error(TBSCI_E_INVAL, "counts is NULL");
        if (nbins < 1 || nbins > 4096) throw Error(TBSCI_E_INVAL, "nbins must be in [1, 4096]");
        if (!(log10_hi > log10_lo)) throw Error(TBSCI_E_INVAL, "need log10_lo < log10_hi");
        hipStream_t st = (hipStream_t)stream;
        const int64_t n = c->dets ? c->dets->n : c->sp[0].l * c->sp[1].l;
        unsigned long long *d = nullptr;
        TB_HIP(hipMalloc((void **)&d, sizeof(unsigned long long) * nbins));
        std::vector<unsigned long long> zero((size_t)nbins, 0ull);
        TB_HIP(hipMemcpyAsync(d, zero.data(), sizeof(unsigned long long) * nbins,
                              hipMemcpyHostToDevice, st));
        const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kB - 1) / kB, 4096));
        k_hist<<<g, kB, sizeof(unsigned int) * nbins, st>>>(n, C_dev, log10_lo, log10_hi, nbins, d);
        TB_HIP(hipGetLastError());
        std::vector<unsigned long long> h((size_t)nbins);
        TB_HIP(hipMemcpyAsync(h.data(), d, sizeof(unsigned long long) * nbins,
                              hipMemcpyDeviceToHost, st));
        TB_HIP(hipStreamSynchronize(st));
        TB_HIP(hipFree(d));
        for (int i = 0; i < nbins; ++i) counts_host[i] = (int64_t)h[(size_t)i];
        return TBSCI_OK;
    });
}

int tbsci_select_strings(tbsci_ctx *ctx, int spin, const double *w_dev, double delta,
                         uint64_t ref_string, uint64_t *out_host, int64_t *n_out, void *stream) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        Ctx *c = ctx_of(ctx);
        if (spin != 0 && spin != 1) throw Error(TBSCI_E_INVAL, "spin must be 0 or 1");
        check_dev(w_dev, c->device, "w");
        if (!out_host || !n_out) throw Error(TBSCI_E_INVAL, "output is NULL");
        if (!(delta >= 0.0)) throw Error(TBSCI_E_INVAL, "delta must be >= 0");
        hipStream_t st = (hipStream_t)stream;
        const Spin &s = c->sp[spin];
        int32_t ref = -1;
        {
            uint64_t *q = nullptr;
            int32_t *r = nullptr;
            TB_HIP(hipMalloc((void **)&q, sizeof(uint64_t)));
            TB_HIP(hipMalloc((void **)&r, sizeof(int32_t)));
            TB_HIP(hipMemcpyAsync(q, &ref_string, sizeof(uint64_t), hipMemcpyHostToDevice, st));
            launch_lookup(s, q, 1, r, st);
            TB_HIP(hipMemcpyAsync(&ref, r, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            TB_HIP(hipStreamSynchronize(st));
            TB_HIP(hipFree(q));
            TB_HIP(hipFree(r));
        }
        if (ref < 0) throw Error(TBSCI_E_INVAL, "the reference string is not in the list");
        std::vector<double> w((size_t)s.l);
        std::vector<uint64_t> str((size_t)s.l);
        TB_HIP(hipMemcpyAsync(w.data(), w_dev, sizeof(double) * s.l, hipMemcpyDeviceToHost, st));
        TB_HIP(hipMemcpyAsync(str.data(), s.str, sizeof(uint64_t) * s.l, hipMemcpyDeviceToHost,
                              st));
        int32_t *flags = nullptr;
        TB_HIP(hipMalloc((void **)&flags, sizeof(int32_t) * std::max<int64_t>(s.l, 1)));
        TB_HIP(hipStreamSynchronize(st));
        const double thresh = delta * w[(size_t)ref];
        k_over<<<(unsigned)((s.l + kB - 1) / kB), kB, 0, st>>>(s.l, w_dev, thresh, flags);
        TB_HIP(hipGetLastError());
        std::vector<int32_t> f((size_t)s.l);
        TB_HIP(hipMemcpyAsync(f.data(), flags, sizeof(int32_t) * s.l, hipMemcpyDeviceToHost, st));
        TB_HIP(hipStreamSynchronize(st));
        TB_HIP(hipFree(flags));
        // the kept strings ranked by weight (heaviest first, ties by the
        // smaller string); the reference string is always kept
        std::vector<int64_t> keep;
        for (int64_t i = 0; i < s.l; ++i)
            if (f[(size_t)i] || i == ref) keep.push_back(i);
        std::sort(keep.begin(), keep.end(), [&](int64_t a, int64_t b) {
            if (w[(size_t)a] != w[(size_t)b]) return w[(size_t)a] > w[(size_t)b];
            return str[(size_t)a] < str[(size_t)b];
        });
        for (size_t k = 0; k < keep.size(); ++k) out_host[k] = str[(size_t)keep[k]];
        *n_out = (int64_t)keep.size();
        return TBSCI_OK;
    });
}

}  // extern "C"
