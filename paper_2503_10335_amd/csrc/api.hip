// C ABI of the TPB sigma library: validation, context lifetime, sigma,
// diagonal and inspection entry points.  Every entry point catches
// exceptions and turns them into status codes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "tbsci_internal.hpp"

namespace tbsci {

thread_local std::string g_err;

namespace {

void check_strings(const char *name, const uint64_t *s, int64_t l, int M, int n) {
    if (!s) throw Error(TBSCI_E_INVAL, std::string(name) + " is NULL");
    if (l < 1 || l > 2147483647LL)
        throw Error(TBSCI_E_INVAL, std::string(name) + ": list length must be in [1, 2^31-1]");
    for (int64_t i = 0; i < l; ++i) {
        if (M < 64 && (s[i] >> M) != 0)
            throw Error(TBSCI_E_INVAL, std::string(name) + ": string " + std::to_string(i) +
                                           " has a bit at or above M");
        if (__builtin_popcountll(s[i]) != n)
            throw Error(TBSCI_E_INVAL, std::string(name) + ": string " + std::to_string(i) +
                                           " has the wrong number of electrons");
    }
    std::vector<uint64_t> v(s, s + l);
    std::sort(v.begin(), v.end());
    if (std::adjacent_find(v.begin(), v.end()) != v.end())
        throw Error(TBSCI_E_INVAL, std::string(name) + ": duplicate strings");
}

void check_integrals(int M, const double *h, const double *eri) {
    if (!h || !eri) throw Error(TBSCI_E_INVAL, "h or eri is NULL");
    double hmax = 0.0, gmax = 0.0;
    const size_t M2 = (size_t)M * M, M4 = M2 * M2;
    for (size_t i = 0; i < M2; ++i) {
        if (!std::isfinite(h[i])) throw Error(TBSCI_E_INVAL, "h has a non-finite entry");
        hmax = std::max(hmax, std::fabs(h[i]));
    }
    for (size_t i = 0; i < M4; ++i) {
        if (!std::isfinite(eri[i])) throw Error(TBSCI_E_INVAL, "eri has a non-finite entry");
        gmax = std::max(gmax, std::fabs(eri[i]));
    }
    const double th = 1e-12 * std::max(1.0, hmax), tg = 1e-12 * std::max(1.0, gmax);
    for (int p = 0; p < M; ++p)
        for (int q = 0; q < M; ++q)
            if (std::fabs(h[p * M + q] - h[q * M + p]) > th)
                throw Error(TBSCI_E_INVAL, "h is not symmetric");
    auto g = [&](int p, int q, int r, int s) { return eri[(((size_t)p * M + q) * M + r) * M + s]; };
    for (int p = 0; p < M; ++p)
        for (int q = 0; q < M; ++q)
            for (int r = 0; r < M; ++r)
                for (int s = 0; s < M; ++s) {
                    const double v = g(p, q, r, s);
                    if (std::fabs(v - g(q, p, r, s)) > tg || std::fabs(v - g(p, q, s, r)) > tg ||
                        std::fabs(v - g(r, s, p, q)) > tg)
                        throw Error(TBSCI_E_INVAL, "eri lacks the 8-fold permutational symmetry");
                }
}

template <typename T>
T *dalloc(size_t n) {
    void *p = nullptr;
    TB_HIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)));
    return (T *)p;
}

void free_spin(Spin &s) {
    free_hole(s);
    void *ptrs[] = {s.str,   s.keys,  s.pos,     s.s_ptr, s.s_ent, s.d_ptr, s.d_ent,
                    s.a_ptr, s.a_col, s.a_val,   s.a_val32, s.dsame, s.jocc,  s.g_ent,
                    s.g_off, s.b_off, s.b_col,   s.b_val, s.b_val32, s.ks_rows};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    s = Spin{};
}

}  // namespace

void destroy_ctx(Ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    timing_clear(*c);
    free_dets(*c);
    for (auto &s : c->sp) free_spin(s);
    void *ptrs[] = {c->h,       c->eri,     c->V64,     c->V32,
                    c->work,    c->det_buf, c->det_stage, c->hole_work};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete c;
}

namespace {

void check_device_ptr(const void *p, int device, const char *name) {
    if (!p) throw Error(TBSCI_E_INVAL, std::string(name) + " is NULL");
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        throw Error(TBSCI_E_INVAL, std::string(name) + " is not a HIP allocation");
    }
    if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
        throw Error(TBSCI_E_INVAL, std::string(name) + " is not device memory");
    if (a.device != device)
        throw Error(TBSCI_E_INVAL, std::string(name) + " is on another device");
}

}  // namespace

Ctx *ctx_of(const tbsci_ctx *p) { return (Ctx *)p; }

void check_ctx(const tbsci_ctx *ctx) {
    if (!ctx) throw Error(TBSCI_E_INVAL, "context is NULL");
    TB_HIP(hipSetDevice(ctx_of(ctx)->device));
}

void check_dev(const void *p, int device, const char *name) { check_device_ptr(p, device, name); }

// sigma on the context's space: the TPB space, or a TBSCI space with
// compact vectors (zero-extended into the context's two dense vectors)
void sigma_any(Ctx &c, const void *C, void *S, int precision, hipStream_t st, int terms) {
    if (!c.dets) {
        launch_sigma(c, C, S, precision, st, terms);
        return;
    }
    const size_t sz = precision == TBSCI_FP64 ? 8 : 4;
    double *X = dets_work(c);
    double *Y = X + c.sp[0].l * c.sp[1].l;
    dets_expand(c, C, X, sz, st);
    launch_sigma(c, X, Y, precision, st, terms);
    dets_gather(c, Y, S, sz, st);
}

}  // namespace tbsci

using namespace tbsci;

extern "C" {

const char *tbsci_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace tbsci {

void validate_problem(int M, int n_alpha, int n_beta, const double *h, const double *eri,
                      const uint64_t *alpha, int64_t l_alpha, const uint64_t *beta,
                      int64_t l_beta) {
    if (M < 1 || M > 64) throw Error(TBSCI_E_INVAL, "M must be in [1, 64]");
    if (n_alpha < 0 || n_alpha > M || n_beta < 0 || n_beta > M)
        throw Error(TBSCI_E_INVAL, "electron counts must be in [0, M]");
    check_strings("alpha", alpha, l_alpha, M, n_alpha);
    check_strings("beta", beta, l_beta, M, n_beta);
    check_integrals(M, h, eri);
}

void check_device_index(int device) {
    int ndev = 0;
    TB_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) throw Error(TBSCI_E_INVAL, "no such device");
}

namespace {

size_t page(size_t bytes) { return (std::max<size_t>(bytes, 8) + 4095) & ~size_t(4095); }

// allocation sizes of one spin's structures (see build_spin), cnt included
size_t spin_bytes(int M, int P, int n, int64_t l, int64_t n_s, int64_t n_d) {
    const size_t L = (size_t)l;
    const int64_t n_a = l + (n_s - (int64_t)n * l) + n_d;
    const size_t ngroup = 4 * (size_t)((P + 15) / 16);
    const int64_t chunk = sweep_chunk(l, n_a);
    const size_t nch = chunk ? (size_t)((l + chunk - 1) / chunk) : 1;
    const size_t chunked = nch > 1 ? page(4 * L * (nch + 1)) + page(4 * (size_t)n_a) +
                                         page(8 * (size_t)n_a) + page(4 * (size_t)n_a)
                                   : 0;
    return page(8 * L) * 2 + page(4 * L) + page(8 * L) + page(8 * (L + 1)) * 3 +
           page(8 * (size_t)n_s) * 2 + page(4 * L * (ngroup + 1)) + page(8 * (size_t)n_d) +
           page(8 * L) + page(8 * L * (size_t)M) + page(4 * (size_t)n_a) +
           page(8 * (size_t)n_a) + page(4 * (size_t)n_a) + chunked;
}

size_t fixed_bytes(int M, int P, int64_t l_alpha, int64_t l_beta) {
    const size_t M2 = (size_t)M * M, PP = (size_t)P * P;
    return page(8 * M2) + page(8 * M2 * M2) + page(8 * PP) + page(4 * PP) +
           page(sigma_work_bytes(l_alpha, l_beta));
}

double binom(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

}  // namespace

size_t ctx_bytes(const Ctx &c) {
    return fixed_bytes(c.M, c.P, c.sp[0].l, c.sp[1].l) +
           spin_bytes(c.M, c.P, c.sp[0].n, c.sp[0].l, c.sp[0].n_s, c.sp[0].n_d) +
           spin_bytes(c.M, c.P, c.sp[1].n, c.sp[1].l, c.sp[1].n_s, c.sp[1].n_d);
}

size_t ctx_bytes_bound(int M, int n_alpha, int n_beta, int64_t l_alpha, int64_t l_beta) {
    const int P = M * (M + 1) / 2;
    size_t b = fixed_bytes(M, P, l_alpha, l_beta);
    const int ns[2] = {n_alpha, n_beta};
    const int64_t ls[2] = {l_alpha, l_beta};
    for (int s = 0; s < 2; ++s) {
        const int n = ns[s];
        const int64_t l = ls[s];
        // each string links to at most l - 1 others, and to at most the
        // complete-space counts n (M - n) singles and C(n,2) C(M-n,2) doubles
        const double s_off = std::min((double)n * (M - n), (double)(l - 1));
        const double d_max = std::min(binom(n, 2) * binom(M - n, 2), (double)(l - 1));
        b += spin_bytes(M, P, n, l, (int64_t)((double)l * (n + s_off)), (int64_t)((double)l * d_max));
    }
    return b;
}

Ctx *create_ctx(int M, int n_alpha, int n_beta, const double *h, const double *eri,
                const uint64_t *alpha, int64_t l_alpha, const uint64_t *beta, int64_t l_beta,
                int device) {
        TB_HIP(hipSetDevice(device));
        Ctx *c = new Ctx();
        try {
            c->M = M;
            c->P = M * (M + 1) / 2;
            c->device = device;
            c->sp[0].n = n_alpha;
            c->sp[0].l = l_alpha;
            c->sp[1].n = n_beta;
            c->sp[1].l = l_beta;
            c->flip_lists = n_alpha == n_beta && l_alpha == l_beta &&
                            std::equal(alpha, alpha + l_alpha, beta);
            c->flip = c->flip_lists;
            const size_t M2 = (size_t)M * M, M4 = M2 * M2, P = c->P;
            std::vector<double> V64(P * P);
            std::vector<float> V32(P * P);
            for (int p = 0; p < M; ++p)
                for (int q = 0; q <= p; ++q)
                    for (int r = 0; r < M; ++r)
                        for (int s = 0; s <= r; ++s) {
                            const double v = eri[(((size_t)p * M + q) * M + r) * M + s];
                            const size_t k = (size_t)fold_pair(p, q) * P + fold_pair(r, s);
                            V64[k] = v;
                            V32[k] = (float)v;
                            c->maxV = std::max(c->maxV, std::fabs(v));
                        }
            hipStream_t st;
            TB_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            try {
                c->h = dalloc<double>(M2);
                c->eri = dalloc<double>(M4);
                c->V64 = dalloc<double>(P * P);
                c->V32 = dalloc<float>(P * P);
                TB_HIP(hipMemcpyAsync(c->h, h, M2 * sizeof(double), hipMemcpyHostToDevice, st));
                TB_HIP(hipMemcpyAsync(c->eri, eri, M4 * sizeof(double), hipMemcpyHostToDevice, st));
                TB_HIP(hipMemcpyAsync(c->V64, V64.data(), P * P * sizeof(double),
                                      hipMemcpyHostToDevice, st));
                TB_HIP(hipMemcpyAsync(c->V32, V32.data(), P * P * sizeof(float),
                                      hipMemcpyHostToDevice, st));
                build_spin(*c, c->sp[0], alpha, st);
                build_spin(*c, c->sp[1], beta, st);
                TB_HIP(hipStreamSynchronize(st));
                build_ks_classes(c->sp[0]);
                // hole-pair index of the spins the automatic method gives it to
                hole_build(*c, 0, false);
                hole_build(*c, 1, false);
            } catch (...) {
                (void)hipStreamSynchronize(st);
                (void)hipStreamDestroy(st);
                throw;
            }
            TB_HIP(hipStreamDestroy(st));
        } catch (...) {
            destroy_ctx(c);
            throw;
        }
        return c;
}

}  // namespace tbsci

extern "C" {

int tbsci_create(int M, int n_alpha, int n_beta, const double *h, const double *eri,
                 const uint64_t *alpha, int64_t l_alpha, const uint64_t *beta, int64_t l_beta,
                 int device, tbsci_ctx **out) {
    return guarded([&]() -> int {
        if (!out) throw Error(TBSCI_E_INVAL, "out is NULL");
        validate_problem(M, n_alpha, n_beta, h, eri, alpha, l_alpha, beta, l_beta);
        check_device_index(device);
        *out = (tbsci_ctx *)create_ctx(M, n_alpha, n_beta, h, eri, alpha, l_alpha, beta, l_beta,
                                       device);
        return TBSCI_OK;
    });
}

void tbsci_destroy(tbsci_ctx *ctx) {
    if (!ctx) return;
    try {
        destroy_ctx(ctx_of(ctx));
    } catch (...) {
    }
}

int tbsci_dims(const tbsci_ctx *ctx, int64_t *l_alpha, int64_t *l_beta, int64_t *n_det) {
    return guarded([&]() -> int {
        if (!ctx) throw Error(TBSCI_E_INVAL, "context is NULL");
        const Ctx *c = ctx_of(ctx);
        if (l_alpha) *l_alpha = c->sp[0].l;
        if (l_beta) *l_beta = c->sp[1].l;
        if (n_det) *n_det = c->dets ? c->dets->n : c->sp[0].l * c->sp[1].l;
        return TBSCI_OK;
    });
}

int tbsci_sigma(tbsci_ctx *ctx, const void *C_dev, void *sigma_dev, int precision, void *stream) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        Ctx *c = ctx_of(ctx);
        if (precision != TBSCI_FP64 && precision != TBSCI_FP32)
            throw Error(TBSCI_E_INVAL, "precision must be TBSCI_FP64 or TBSCI_FP32");
        check_dev(C_dev, c->device, "C");
        check_dev(sigma_dev, c->device, "sigma");
        if (C_dev == sigma_dev) throw Error(TBSCI_E_INVAL, "C and sigma must not alias");
        sigma_any(*c, C_dev, sigma_dev, precision, (hipStream_t)stream, 7);
        return TBSCI_OK;
    });
}

int tbsci_sigma_terms(tbsci_ctx *ctx, const void *C_dev, void *sigma_dev, int precision,
                      int terms, void *stream) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        Ctx *c = ctx_of(ctx);
        if (precision != TBSCI_FP64 && precision != TBSCI_FP32)
            throw Error(TBSCI_E_INVAL, "precision must be TBSCI_FP64 or TBSCI_FP32");
        if (terms < 0 || terms > 7) throw Error(TBSCI_E_INVAL, "terms must be a mask in 0..7");
        check_dev(C_dev, c->device, "C");
        check_dev(sigma_dev, c->device, "sigma");
        if (C_dev == sigma_dev) throw Error(TBSCI_E_INVAL, "C and sigma must not alias");
        sigma_any(*c, C_dev, sigma_dev, precision, (hipStream_t)stream, terms);
        return TBSCI_OK;
    });
}

int tbsci_diag(tbsci_ctx *ctx, double *diag_dev, void *stream) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        Ctx *c = ctx_of(ctx);
        check_dev(diag_dev, c->device, "diag");
        if (c->dets) {  // H_KK of the kept determinants, compact
            double *X = dets_work(*c);
            launch_full_diag(*c, X, (hipStream_t)stream);
            dets_gather(*c, X, diag_dev, 8, (hipStream_t)stream);
        } else {
            launch_full_diag(*c, diag_dev, (hipStream_t)stream);
        }
        return TBSCI_OK;
    });
}

int tbsci_string_index(const tbsci_ctx *ctx, int spin, uint64_t *keys_host, int32_t *pos_host) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        if (spin != 0 && spin != 1) throw Error(TBSCI_E_INVAL, "spin must be 0 or 1");
        if (!keys_host || !pos_host) throw Error(TBSCI_E_INVAL, "output is NULL");
        const Spin &s = ctx_of(ctx)->sp[spin];
        TB_HIP(hipMemcpy(keys_host, s.keys, s.l * sizeof(uint64_t), hipMemcpyDeviceToHost));
        TB_HIP(hipMemcpy(pos_host, s.pos, s.l * sizeof(int32_t), hipMemcpyDeviceToHost));
        return TBSCI_OK;
    });
}

int tbsci_lookup(const tbsci_ctx *ctx, int spin, const uint64_t *queries_dev, int64_t n,
                 int32_t *out_dev, void *stream) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        if (spin != 0 && spin != 1) throw Error(TBSCI_E_INVAL, "spin must be 0 or 1");
        if (n < 0) throw Error(TBSCI_E_INVAL, "n < 0");
        if (n == 0) return TBSCI_OK;
        const Ctx *c = ctx_of(ctx);
        check_dev(queries_dev, c->device, "queries");
        check_dev(out_dev, c->device, "out");
        launch_lookup(c->sp[spin], queries_dev, n, out_dev, (hipStream_t)stream);
        return TBSCI_OK;
    });
}

int tbsci_list_size(const tbsci_ctx *ctx, int spin, int kind, int64_t *n_entries) {
    return guarded([&]() -> int {
        if (!ctx) throw Error(TBSCI_E_INVAL, "context is NULL");
        if (spin != 0 && spin != 1) throw Error(TBSCI_E_INVAL, "spin must be 0 or 1");
        if (!n_entries) throw Error(TBSCI_E_INVAL, "n_entries is NULL");
        const Spin &s = ctx_of(ctx)->sp[spin];
        if (kind == 1)
            *n_entries = s.n_s;
        else if (kind == 2)
            *n_entries = s.n_d;
        else if (kind == 3)
            *n_entries = s.n_a;
        else
            throw Error(TBSCI_E_INVAL, "kind must be 1, 2 or 3");
        return TBSCI_OK;
    });
}

int tbsci_get_list(const tbsci_ctx *ctx, int spin, int kind, int64_t *row_ptr_host,
                   int32_t *entries_host, double *values_host) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        if (spin != 0 && spin != 1) throw Error(TBSCI_E_INVAL, "spin must be 0 or 1");
        if (kind < 1 || kind > 3) throw Error(TBSCI_E_INVAL, "kind must be 1, 2 or 3");
        if (!row_ptr_host || !entries_host || (kind == 3 && !values_host))
            throw Error(TBSCI_E_INVAL, "output is NULL");
        const Spin &s = ctx_of(ctx)->sp[spin];
        const int64_t *ptr = kind == 1 ? s.s_ptr : kind == 2 ? s.d_ptr : s.a_ptr;
        const int64_t n = kind == 1 ? s.n_s : kind == 2 ? s.n_d : s.n_a;
        TB_HIP(hipMemcpy(row_ptr_host, ptr, (s.l + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
        if (kind == 3) {
            TB_HIP(hipMemcpy(entries_host, s.a_col, n * sizeof(int32_t), hipMemcpyDeviceToHost));
            TB_HIP(hipMemcpy(values_host, s.a_val, n * sizeof(double), hipMemcpyDeviceToHost));
            return TBSCI_OK;
        }
        std::vector<Ent> e(std::max<int64_t>(n, 1));
        TB_HIP(hipMemcpy(e.data(), kind == 1 ? s.s_ent : s.d_ent, n * sizeof(Ent),
                         hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i) {
            int32_t *o = entries_host + 6 * i;
            const uint32_t w = e[i].o;
            o[0] = e[i].j;
            if (kind == 1) {
                o[1] = w & 63;
                o[2] = (w >> 6) & 63;
                o[3] = o[4] = 0;
                o[5] = ((w >> 12) & 1) ? -1 : 1;
            } else {
                o[1] = w & 63;
                o[2] = (w >> 6) & 63;
                o[3] = (w >> 12) & 63;
                o[4] = (w >> 18) & 63;
                o[5] = ((w >> 24) & 1) ? -1 : 1;
            }
        }
        return TBSCI_OK;
    });
}

int tbsci_timing_enable(tbsci_ctx *ctx, int enable) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        Ctx *c = ctx_of(ctx);
        timing_clear(*c);
        c->timing = enable != 0;
        return TBSCI_OK;
    });
}

int tbsci_set_deterministic(tbsci_ctx *ctx, int enable) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        Ctx *c = ctx_of(ctx);
        if (enable) {
            TB_HIP(hipSetDevice(c->device));
            if (!c->det_buf) c->det_buf = dalloc<double>(2);
            const int64_t n = det_stage_entries(*c);
            if (n > c->det_stage_n) {
                if (c->det_stage) TB_HIP(hipFree(c->det_stage));
                c->det_stage = nullptr;
                c->det_stage_n = 0;
                c->det_stage = dalloc<unsigned long long>((size_t)n);
                TB_HIP(hipMemset(c->det_stage, 0, (size_t)n * 8));
                c->det_stage_n = n;
            }
        }
        c->det = enable != 0;
        return TBSCI_OK;
    });
}

int tbsci_set_same_spin(tbsci_ctx *ctx, int method) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        Ctx *c = ctx_of(ctx);
        if (method != TBSCI_SAME_SPIN_AUTO && method != TBSCI_SAME_SPIN_CSR &&
            method != TBSCI_SAME_SPIN_HOLE)
            throw Error(TBSCI_E_INVAL, "unknown same-spin method");
        if (method != TBSCI_SAME_SPIN_CSR) {
            TB_HIP(hipSetDevice(c->device));
            hole_build(*c, 0, method == TBSCI_SAME_SPIN_HOLE);
            hole_build(*c, 1, method == TBSCI_SAME_SPIN_HOLE);
        }
        c->same_spin = method;
        return TBSCI_OK;
    });
}

int tbsci_timing_read(tbsci_ctx *ctx, int kernel, int precision, double *total_ms,
                      int64_t *launches, double *flops, double *bytes, const char **name) {
    static const char *names[TBSCI_N_KERNELS] = {"same_spin_alpha_sweep", "same_spin_beta_sweep",
                                                 "opposite_spin"};
    return guarded([&]() -> int {
        check_ctx(ctx);
        if (kernel < 0 || kernel >= TBSCI_N_KERNELS) throw Error(TBSCI_E_INVAL, "no such kernel");
        if (precision != TBSCI_FP64 && precision != TBSCI_FP32)
            throw Error(TBSCI_E_INVAL, "precision must be TBSCI_FP64 or TBSCI_FP32");
        Ctx *c = ctx_of(ctx);
        double ms = 0.0;
        int64_t n = 0;
        for (auto &t : c->timed) {
            if (t.precision != precision) continue;
            TB_HIP(hipEventSynchronize(t.ev[kernel + 1]));
            float x = 0.f;
            TB_HIP(hipEventElapsedTime(&x, t.ev[kernel], t.ev[kernel + 1]));
            ms += x;
            ++n;
        }
        const Spin &A = c->sp[0], &B = c->sp[1];
        const double la = (double)A.l, lb = (double)B.l, nd = la * lb;
        const double sz = precision == TBSCI_FP64 ? 8.0 : 4.0;
        double f = 0.0, b = 0.0;
        if (kernel == 0) {
            f = 2.0 * (double)A.n_a * lb;
            b = 2.0 * nd * sz + 8.0 * (la + 1) + (4.0 + sz) * (double)A.n_a;
        } else if (kernel == 1) {
            f = 2.0 * (double)B.n_a * la;
            b = 3.0 * nd * sz + 8.0 * (lb + 1) + (4.0 + sz) * (double)B.n_a;
        } else {
            f = 2.0 * (double)A.n_s * (double)B.n_s;
            b = 3.0 * nd * sz + 8.0 * (la + lb + 2) + 8.0 * (double)(A.n_s + B.n_s) +
                sz * (double)c->P * c->P;
        }
        if (total_ms) *total_ms = ms;
        if (launches) *launches = n;
        if (flops) *flops = f;
        if (bytes) *bytes = b;
        if (name) *name = names[kernel];
        return TBSCI_OK;
    });
}

int tbsci_timing_executed_flops(tbsci_ctx *ctx, int kernel, int precision, double *flops) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        if (kernel < 0 || kernel >= TBSCI_N_KERNELS) throw Error(TBSCI_E_INVAL, "no such kernel");
        if (precision != TBSCI_FP64 && precision != TBSCI_FP32)
            throw Error(TBSCI_E_INVAL, "precision must be TBSCI_FP64 or TBSCI_FP32");
        if (!flops) throw Error(TBSCI_E_INVAL, "flops is NULL");
        *flops = executed_flops(*ctx_of(ctx), kernel, precision);
        return TBSCI_OK;
    });
}

}  // extern "C"
