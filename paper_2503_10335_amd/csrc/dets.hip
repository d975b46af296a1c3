// TBSCI spaces: determinant-level pruning of the TPB space (paper Sec. II.A:
// per alpha string w the index set I_w of the beta strings it is paired
// with; segments of the CI vector have their own offsets and lengths).
//
// The boundary takes compact vectors -- the kept determinants, row w's
// segment after row w-1's, each segment in ascending beta index.  sigma =
// P H P C restricted to the space equals the TPB sigma of the vector
// extended by zeros, read at the kept determinants, because the projector is
// diagonal in the TPB basis: the membership of the output determinant
// (u in I_w) is the read-back, that of every contributing one (v in I_x,
// Algorithm 1) the zeros.  So the sigma kernels stay those of the TPB space;
// a TBSCI space costs the TPB space's work plus two zero-extended vectors.
#include <algorithm>

#include "tbsci_internal.hpp"

namespace tbsci {
namespace {

constexpr int kB = 256;

// one block per alpha row: dense[w][idx[k]] = compact[k] for k in row w's
// segment (dense zeroed before)
template <typename T>
__global__ __launch_bounds__(kB) void k_expand(int64_t lb, const int64_t *__restrict__ off,
                                               const int32_t *__restrict__ idx,
                                               const T *__restrict__ c, T *__restrict__ d) {
    const int64_t w = blockIdx.x;
    const int64_t k1 = off[w + 1];
    for (int64_t k = off[w] + threadIdx.x; k < k1; k += kB) d[w * lb + idx[k]] = c[k];
}

template <typename T>
__global__ __launch_bounds__(kB) void k_gather(int64_t lb, const int64_t *__restrict__ off,
                                               const int32_t *__restrict__ idx,
                                               const T *__restrict__ d, T *__restrict__ c) {
    const int64_t w = blockIdx.x;
    const int64_t k1 = off[w + 1];
    for (int64_t k = off[w] + threadIdx.x; k < k1; k += kB) c[k] = d[w * lb + idx[k]];
}

template <typename T>
__global__ __launch_bounds__(kB) void k_fill0(int64_t n, T *__restrict__ o) {
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
        o[i] = T(0);
}

// d[w][u] = 0 unless bit u of mask row w is set
__global__ __launch_bounds__(kB) void k_mask(int64_t la, int64_t lb, int64_t wpr,
                                             const uint32_t *__restrict__ m,
                                             double *__restrict__ d) {
    const int64_t n = la * lb;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kB) {
        const int64_t w = i / lb, u = i - w * lb;
        if (!((m[w * wpr + (u >> 5)] >> (u & 31)) & 1u)) d[i] = 0.0;
    }
}

unsigned grid_for(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kB - 1) / kB, 16384));
}

}  // namespace

void free_dets(Ctx &c) {
    if (!c.dets) return;
    void *ptrs[] = {c.dets->off, c.dets->idx, c.dets->mask, c.dets->work};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete c.dets;
    c.dets = nullptr;
}

void dets_expand(Ctx &c, const void *compact, void *dense, size_t sz, hipStream_t st) {
    const int64_t la = c.sp[0].l, lb = c.sp[1].l;
    if (sz == 8) {
        k_fill0<double><<<grid_for(la * lb), kB, 0, st>>>(la * lb, (double *)dense);
        k_expand<double><<<(unsigned)la, kB, 0, st>>>(lb, c.dets->off, c.dets->idx,
                                                      (const double *)compact, (double *)dense);
    } else {
        k_fill0<float><<<grid_for(la * lb), kB, 0, st>>>(la * lb, (float *)dense);
        k_expand<float><<<(unsigned)la, kB, 0, st>>>(lb, c.dets->off, c.dets->idx,
                                                     (const float *)compact, (float *)dense);
    }
    TB_HIP(hipGetLastError());
}

void dets_gather(Ctx &c, const void *dense, void *compact, size_t sz, hipStream_t st) {
    const int64_t la = c.sp[0].l, lb = c.sp[1].l;
    if (sz == 8)
        k_gather<double><<<(unsigned)la, kB, 0, st>>>(lb, c.dets->off, c.dets->idx,
                                                      (const double *)dense, (double *)compact);
    else
        k_gather<float><<<(unsigned)la, kB, 0, st>>>(lb, c.dets->off, c.dets->idx,
                                                     (const float *)dense, (float *)compact);
    TB_HIP(hipGetLastError());
}

void dets_mask(Ctx &c, double *dense, hipStream_t st) {
    const int64_t la = c.sp[0].l, lb = c.sp[1].l;
    k_mask<<<grid_for(la * lb), kB, 0, st>>>(la, lb, c.dets->wpr, c.dets->mask, dense);
    TB_HIP(hipGetLastError());
}

double *dets_work(Ctx &c) {
    Dets &d = *c.dets;
    const size_t need = 2 * sizeof(double) * (size_t)(c.sp[0].l * c.sp[1].l);
    if (d.work_bytes < need) {
        if (d.work) TB_HIP(hipFree(d.work));
        d.work = nullptr;
        d.work_bytes = 0;
        TB_HIP(hipMalloc(&d.work, need));
        d.work_bytes = need;
    }
    return (double *)d.work;
}

}  // namespace tbsci

using namespace tbsci;

extern "C" {

int tbsci_set_dets(tbsci_ctx *ctx, const int64_t *row_off, const int32_t *beta_idx) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        Ctx *c = ctx_of(ctx);
        if (!row_off && !beta_idx) {  // back to the whole TPB space
            free_dets(*c);
            c->flip = c->flip_lists;
            return TBSCI_OK;
        }
        install_dets(*c, row_off, beta_idx);
        return TBSCI_OK;
    });
}

int tbsci_get_dets(const tbsci_ctx *ctx, int64_t *row_off_host, int32_t *beta_idx_host) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        const Ctx *c = ctx_of(ctx);
        if (!c->dets) throw Error(TBSCI_E_STATE, "the context has no TBSCI space");
        if (!row_off_host || !beta_idx_host) throw Error(TBSCI_E_INVAL, "output is NULL");
        TB_HIP(hipMemcpy(row_off_host, c->dets->off, sizeof(int64_t) * (c->sp[0].l + 1),
                         hipMemcpyDeviceToHost));
        TB_HIP(hipMemcpy(beta_idx_host, c->dets->idx, sizeof(int32_t) * c->dets->n,
                         hipMemcpyDeviceToHost));
        return TBSCI_OK;
    });
}

}  // extern "C"

namespace tbsci {

void install_dets(Ctx &cc, const int64_t *row_off, const int32_t *beta_idx) {
    {
        Ctx *c = &cc;
        const int64_t la = c->sp[0].l, lb = c->sp[1].l;
        if (!row_off || !beta_idx) throw Error(TBSCI_E_INVAL, "row_off or beta_idx is NULL");
        if (row_off[0] != 0) throw Error(TBSCI_E_INVAL, "row_off[0] must be 0");
        for (int64_t w = 0; w < la; ++w) {
            if (row_off[w + 1] < row_off[w] || row_off[w + 1] - row_off[w] > lb)
                throw Error(TBSCI_E_INVAL, "row_off must be nondecreasing with at most l_beta "
                                           "entries per row");
            for (int64_t k = row_off[w]; k < row_off[w + 1]; ++k) {
                if (beta_idx[k] < 0 || beta_idx[k] >= lb)
                    throw Error(TBSCI_E_INVAL, "beta_idx outside [0, l_beta)");
                if (k > row_off[w] && beta_idx[k] <= beta_idx[k - 1])
                    throw Error(TBSCI_E_INVAL, "beta_idx must ascend within a row");
            }
        }
        const int64_t n = row_off[la];
        if (n < 1) throw Error(TBSCI_E_INVAL, "the space keeps no determinant");
        const int64_t wpr = (lb + 31) / 32;
        std::vector<uint32_t> mask((size_t)(la * wpr), 0u);
        for (int64_t w = 0; w < la; ++w)
            for (int64_t k = row_off[w]; k < row_off[w + 1]; ++k)
                mask[(size_t)(w * wpr + (beta_idx[k] >> 5))] |= 1u << (beta_idx[k] & 31);
        bool sym = la == lb;
        for (int64_t w = 0; sym && w < la; ++w)
            for (int64_t k = row_off[w]; sym && k < row_off[w + 1]; ++k) {
                const int64_t u = beta_idx[k];
                sym = (mask[(size_t)(u * wpr + (w >> 5))] >> (w & 31)) & 1u;
            }
        bool open = false;
        for (int64_t w = 0; !open && w < la; ++w)
            for (int64_t k = row_off[w]; !open && k < row_off[w + 1]; ++k) open = beta_idx[k] != w;
        auto *d = new Dets();
        try {
            d->n = n;
            d->wpr = wpr;
            d->symmetric = sym;
            d->open_pairs = open;
            TB_HIP(hipMalloc((void **)&d->off, sizeof(int64_t) * (la + 1)));
            TB_HIP(hipMalloc((void **)&d->idx, sizeof(int32_t) * n));
            TB_HIP(hipMalloc((void **)&d->mask, sizeof(uint32_t) * mask.size()));
            TB_HIP(hipMemcpy(d->off, row_off, sizeof(int64_t) * (la + 1), hipMemcpyHostToDevice));
            TB_HIP(hipMemcpy(d->idx, beta_idx, sizeof(int32_t) * n, hipMemcpyHostToDevice));
            TB_HIP(hipMemcpy(d->mask, mask.data(), sizeof(uint32_t) * mask.size(),
                             hipMemcpyHostToDevice));
        } catch (...) {
            Ctx tmp;
            tmp.dets = d;
            free_dets(tmp);
            throw;
        }
        free_dets(*c);
        c->dets = d;
        // the spin flip maps the space onto itself only when it is symmetric
        c->flip = c->flip_lists && sym;
    }
}

}  // namespace tbsci
