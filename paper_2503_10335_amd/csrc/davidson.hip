// Davidson solver for the lowest eigenpair of P H P (paper Sec. II.B: the
// Davidson diagonalisation whose dominant cost is the sigma product;
// Sec. III.C: a restart scheme that bounds the number of stored vectors;
// Sec. III.A: a single-precision matrix-vector product with everything else
// in double precision).
//
// All vector arithmetic runs on the device in FP64: two-pass Gram-Schmidt,
// the new column of the projected matrix V^T H V, the Ritz vector, the
// residual and the diagonal preconditioner.  Only k x k scalars cross to the
// host, where the projected eigenproblem is solved by cyclic Jacobi.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "tbsci_internal.hpp"

namespace tbsci {

namespace {

constexpr int kB = 256;
constexpr int kRedBlocks = 512;  // fixed partial count: deterministic reductions
constexpr int kMaxVec = 64;

struct VecList {
    const double *p[kMaxVec];
};

// partial[i][blk] = sum over this block's slice of a[i] . b
__global__ __launch_bounds__(kB) void k_multidot(int64_t n, VecList a, int k,
                                                 const double *__restrict__ b,
                                                 double *__restrict__ partial) {
    __shared__ double red[kB];
    for (int i = 0; i < k; ++i) {
        const double *__restrict__ ai = a.p[i];
        double s = 0.0;
        for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t < n; t += (int64_t)gridDim.x * kB)
            s += ai[t] * b[t];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int off = kB / 2; off > 0; off >>= 1) {
            if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[i * gridDim.x + blockIdx.x] = red[0];
        __syncthreads();
    }
}

// out[i] = sum_blk partial[i][blk], one block per i
__global__ __launch_bounds__(kB) void k_reduce(const double *__restrict__ partial, int nblk,
                                               double *__restrict__ out) {
    __shared__ double red[kB];
    double s = 0.0;
    for (int t = threadIdx.x; t < nblk; t += kB) s += partial[blockIdx.x * nblk + t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = kB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// t -= sum_i coef[i] * a[i]
__global__ __launch_bounds__(kB) void k_sub_proj(int64_t n, VecList a, int k,
                                                 const double *__restrict__ coef,
                                                 double *__restrict__ t) {
    for (int64_t x = (int64_t)blockIdx.x * kB + threadIdx.x; x < n; x += (int64_t)gridDim.x * kB) {
        double v = t[x];
        for (int i = 0; i < k; ++i) v -= coef[i] * a.p[i][x];
        t[x] = v;
    }
}

__global__ __launch_bounds__(kB) void k_scale_by_rnorm(int64_t n, const double *__restrict__ nrm2,
                                                       double *__restrict__ t) {
    const double s = 1.0 / sqrt(nrm2[0]);
    for (int64_t x = (int64_t)blockIdx.x * kB + threadIdx.x; x < n; x += (int64_t)gridDim.x * kB)
        t[x] *= s;
}

// x = V y, wx = W y, r = wx - theta x, t = r / (theta - H_KK) with a floor;
// partial sums of |r|^2.  H_KK is rebuilt from the per-string parts.
__global__ __launch_bounds__(kB) void k_ritz(int64_t n, int64_t lb, int M, VecList V, VecList W,
                                             int k, const double *__restrict__ y, double theta,
                                             double floor_, const uint64_t *__restrict__ astr,
                                             const double *__restrict__ da,
                                             const double *__restrict__ db,
                                             const double *__restrict__ jb, double *__restrict__ xo,
                                             double *__restrict__ wxo, double *__restrict__ to,
                                             double *__restrict__ partial) {
    __shared__ double red[kB];
    double s = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t < n; t += (int64_t)gridDim.x * kB) {
        double xv = 0.0, wv = 0.0;
        for (int i = 0; i < k; ++i) {
            xv += y[i] * V.p[i][t];
            wv += y[i] * W.p[i][t];
        }
        const double r = wv - theta * xv;
        s += r * r;
        const int64_t ia = t / lb, ib = t - ia * lb;
        double d = da[ia] + db[ib];
        const double *jr = jb + ib * M;
        for (uint64_t m = astr[ia]; m; m &= m - 1) d += jr[__builtin_ctzll(m)];
        double den = theta - d;
        if (fabs(den) < floor_) den = den < 0.0 ? -floor_ : floor_;
        xo[t] = xv;
        wxo[t] = wv;
        to[t] = r / den;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = kB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// xo = sum_i z[i] V[i], wo = sum_i z[i] W[i]
__global__ __launch_bounds__(kB) void k_lincomb2(int64_t n, VecList V, VecList W, int k,
                                                 const double *__restrict__ z,
                                                 double *__restrict__ xo,
                                                 double *__restrict__ wo) {
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t < n; t += (int64_t)gridDim.x * kB) {
        double xv = 0.0, wv = 0.0;
        for (int i = 0; i < k; ++i) {
            xv += z[i] * V.p[i][t];
            wv += z[i] * W.p[i][t];
        }
        xo[t] = xv;
        wo[t] = wv;
    }
}

// v = e_at, or (e_at + e_at2) / sqrt(2) when at2 != at
__global__ void k_unit(int64_t n, int64_t at, int64_t at2, double *__restrict__ v) {
    const double val = at2 == at ? 1.0 : 0.70710678118654752440;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        v[x] = (x == at || x == at2) ? val : 0.0;
}

__global__ __launch_bounds__(kB) void k_flip_sym(int64_t l, double *__restrict__ T) {
    flip_sym_block(blockIdx.x, l, T);
}

__global__ void k_to_f32(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        b[x] = (float)a[x];
}

__global__ void k_to_f64(int64_t n, const float *__restrict__ a, double *__restrict__ b) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        b[x] = (double)a[x];
}

// per-block (max |v|, first index)
__global__ __launch_bounds__(kB) void k_absmax(int64_t n, const double *__restrict__ v,
                                               double *__restrict__ pv, int64_t *__restrict__ pi) {
    __shared__ double sv[kB];
    __shared__ int64_t si[kB];
    double best = -1.0;
    int64_t bi = -1;
    for (int64_t x = (int64_t)blockIdx.x * kB + threadIdx.x; x < n; x += (int64_t)gridDim.x * kB) {
        const double a = fabs(v[x]);
        if (a > best) {
            best = a;
            bi = x;
        }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int off = kB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            const double b2 = sv[threadIdx.x + off];
            const int64_t i2 = si[threadIdx.x + off];
            if (b2 > sv[threadIdx.x] || (b2 == sv[threadIdx.x] && i2 >= 0 &&
                                         (si[threadIdx.x] < 0 || i2 < si[threadIdx.x]))) {
                sv[threadIdx.x] = b2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pv[blockIdx.x] = sv[0];
        pi[blockIdx.x] = si[0];
    }
}

__global__ void k_scale_const(int64_t n, double s, double *__restrict__ v) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        v[x] *= s;
}

}  // namespace

// Cyclic Jacobi on a symmetric k x k matrix: eigenvalues w, eigenvectors
// in the columns of Z (row-major k x k).
void jacobi_eigh(int k, std::vector<double> A, std::vector<double> &w, std::vector<double> &Z) {
    Z.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) Z[i * k + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                tot += A[i * k + j] * A[i * k + j];
                if (i != j) off += A[i * k + j] * A[i * k + j];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < k; ++p)
            for (int q = p + 1; q < k; ++q) {
                const double apq = A[p * k + q];
                if (apq == 0.0) continue;
                const double app = A[p * k + p], aqq = A[q * k + q];
                const double tau = (aqq - app) / (2.0 * apq);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int r = 0; r < k; ++r) {  // A = J^T A J
                    const double arp = A[r * k + p], arq = A[r * k + q];
                    A[r * k + p] = c * arp - s * arq;
                    A[r * k + q] = s * arp + c * arq;
                }
                for (int r = 0; r < k; ++r) {
                    const double apr = A[p * k + r], aqr = A[q * k + r];
                    A[p * k + r] = c * apr - s * aqr;
                    A[q * k + r] = s * apr + c * aqr;
                }
                for (int r = 0; r < k; ++r) {
                    const double zrp = Z[r * k + p], zrq = Z[r * k + q];
                    Z[r * k + p] = c * zrp - s * zrq;
                    Z[r * k + q] = s * zrp + c * zrq;
                }
            }
    }
    w.resize(k);
    for (int i = 0; i < k; ++i) w[i] = A[i * k + i];
}

namespace {

struct Workspace {
    std::vector<double *> bufs;
    ~Workspace() {
        for (double *p : bufs)
            if (p) (void)hipFree(p);
    }
    double *get(size_t n) {
        void *p = nullptr;
        TB_HIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(double)));
        bufs.push_back((double *)p);
        return (double *)p;
    }
};

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    Events() {
        TB_HIP(hipEventCreate(&a));
        TB_HIP(hipEventCreate(&b));
    }
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

// Shared by the serving engine: one solve on an existing context.
size_t davidson_bytes(int64_t n, const tbsci_davidson_opts &o) {
    auto page = [](size_t b) { return (std::max<size_t>(b, 8) + 4095) & ~size_t(4095); };
    size_t b = (size_t)(2 * o.n_max + 5) * page(8 * (size_t)n);
    if (o.precision == TBSCI_MIXED) b += 2 * page(8 * (size_t)((n + 1) / 2));
    b += page(8 * (size_t)kMaxVec * kRedBlocks) + 2 * page(8 * (size_t)kMaxVec) +
         page(8 * (size_t)kRedBlocks);
    return b;
}

int davidson_run(Ctx &c, const tbsci_davidson_opts &o, const double *guess, double *C_out,
                 tbsci_davidson_info &info, hipStream_t st, const std::atomic<bool> *abort) {
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t la = c.sp[0].l, lb = c.sp[1].l, n = la * lb;
    const int nmax = o.n_max;
    const bool mixed = o.precision == TBSCI_MIXED;
    const unsigned gb = (unsigned)std::min<int64_t>(kRedBlocks, (n + kB - 1) / kB);
    Workspace ws;
    std::vector<double *> V(nmax), W(nmax);
    for (int i = 0; i < nmax; ++i) {
        V[i] = ws.get(n);
        W[i] = ws.get(n);
    }
    double *X = ws.get(n), *WX = ws.get(n), *T = ws.get(n);
    double *XP = ws.get(n), *WXP = ws.get(n);  // previous Ritz direction for the restart
    float *T32 = nullptr, *S32 = nullptr;
    if (mixed) {
        T32 = (float *)ws.get((n + 1) / 2);
        S32 = (float *)ws.get((n + 1) / 2);
    }
    double *partial = ws.get((size_t)kMaxVec * kRedBlocks);
    double *dots = ws.get(kMaxVec);
    double *ydev = ws.get(kMaxVec);
    int64_t *pidx = (int64_t *)ws.get(kRedBlocks);
    Events ev;

    memset(&info, 0, sizeof(info));
    // flip-symmetric space and no guess: the solve is kept in the C = C^T
    // sector (start vector symmetric, every correction symmetrised), so that
    // rounding in the sigma build cannot carry it into the other sector
    const bool sym = c.flip && !guess;
    const char *tr_env = getenv("TBSCI_DAVIDSON_TRACE");  // per-iteration trace on stderr
    const bool trace = tr_env && tr_env[0] && tr_env[0] != '0';
    double t_sigma = 0.0;
    bool fp32 = mixed;
    auto sigma = [&](const double *in, double *out) {
        TB_HIP(hipEventRecord(ev.a, st));
        if (fp32) {
            k_to_f32<<<1024, kB, 0, st>>>(n, in, T32);
            launch_sigma(c, T32, S32, TBSCI_FP32, st);
            k_to_f64<<<1024, kB, 0, st>>>(n, S32, out);
            info.iters_fp32++;
        } else {
            launch_sigma(c, in, out, TBSCI_FP64, st);
            info.iters_fp64++;
        }
        TB_HIP(hipEventRecord(ev.b, st));
        TB_HIP(hipEventSynchronize(ev.b));
        float ms = 0.f;
        TB_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
        t_sigma += ms * 1e-3;
        info.iters++;
    };
    auto vl = [&](const std::vector<double *> &v, int k) {
        VecList L{};
        for (int i = 0; i < k; ++i) L.p[i] = v[i];
        return L;
    };
    // dots[0..k) = a[i] . b  (device), optionally copied to host
    auto multidot = [&](const std::vector<double *> &a, int k, const double *b, double *host) {
        k_multidot<<<gb, kB, 0, st>>>(n, vl(a, k), k, b, partial);
        k_reduce<<<k, kB, 0, st>>>(partial, gb, dots);
        TB_HIP(hipGetLastError());
        if (host) {
            TB_HIP(hipMemcpyAsync(host, dots, k * sizeof(double), hipMemcpyDeviceToHost, st));
            TB_HIP(hipStreamSynchronize(st));
        }
    };

    // initial vector
    if (guess) {
        TB_HIP(hipMemcpyAsync(V[0], guess, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        double nn;
        std::vector<double *> one{V[0]};
        multidot(one, 1, V[0], &nn);
        if (!(nn > 0.0)) throw Error(TBSCI_E_INVAL, "guess vector is zero");
        k_scale_by_rnorm<<<1024, kB, 0, st>>>(n, dots, V[0]);
    } else {
        launch_diag_argmin(c, partial, pidx, kRedBlocks, st);
        std::vector<double> pv(kRedBlocks);
        std::vector<int64_t> pi(kRedBlocks);
        TB_HIP(hipMemcpyAsync(pv.data(), partial, kRedBlocks * sizeof(double), hipMemcpyDeviceToHost, st));
        TB_HIP(hipMemcpyAsync(pi.data(), pidx, kRedBlocks * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        TB_HIP(hipStreamSynchronize(st));
        double best = 1e308;
        int64_t at = 0;
        for (int b = 0; b < kRedBlocks; ++b)
            if (pi[b] >= 0 && (pv[b] < best || (pv[b] == best && pi[b] < at))) {
                best = pv[b];
                at = pi[b];
            }
        // in a flip-symmetric space an open-shell start |I J> becomes
        // (|I J> + |J I>) / sqrt(2), so the solve stays in the C = C^T sector
        const int64_t ia = at / lb, ib = at - ia * lb;
        const int64_t at2 = c.flip ? ib * lb + ia : at;
        k_unit<<<1024, kB, 0, st>>>(n, at, at2, V[0]);
    }
    TB_HIP(hipGetLastError());

    std::vector<double> G((size_t)nmax * nmax, 0.0), col(kMaxVec), w, Z, yprev;
    int k = 1;
    sigma(V[0], W[0]);
    multidot(V, 1, W[0], col.data());
    G[0] = col[0];
    double theta = 0.0, theta_prev = 0.0, rn = 1e300, best_rn = 1e300;
    int since_best = 0;
    bool done = false, converged = false, force_fp64 = false;
    while (!done) {
        std::vector<double> Gk((size_t)k * k);
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) Gk[i * k + j] = 0.5 * (G[i * nmax + j] + G[j * nmax + i]);
        jacobi_eigh(k, Gk, w, Z);
        int lo = 0;
        for (int i = 1; i < k; ++i)
            if (w[i] < w[lo]) lo = i;
        theta_prev = theta;
        theta = w[lo];
        std::vector<double> y(k);
        for (int i = 0; i < k; ++i) y[i] = Z[i * k + lo];
        std::vector<double> yp = yprev;  // previous Ritz coefficients in this basis
        yp.resize(k, 0.0);
        yprev = y;
        TB_HIP(hipMemcpyAsync(ydev, y.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
        k_ritz<<<gb, kB, 0, st>>>(n, lb, c.M, vl(V, k), vl(W, k), k, ydev, theta, o.precond_floor,
                                  c.sp[0].str, c.sp[0].dsame, c.sp[1].dsame, c.sp[1].jocc, X, WX, T,
                                  partial);
        k_reduce<<<1, kB, 0, st>>>(partial, gb, dots);
        if (sym) {
            const int64_t nt = (lb + 31) / 32;
            k_flip_sym<<<(unsigned)(nt * nt), kB, 0, st>>>(lb, T);
        }
        double r2;
        TB_HIP(hipMemcpyAsync(&r2, dots, sizeof(double), hipMemcpyDeviceToHost, st));
        TB_HIP(hipStreamSynchronize(st));
        rn = std::sqrt(std::max(r2, 0.0));
        if (trace)
            fprintf(stderr, "tbsci davidson: sigma %d k %d %s theta %.15f resid %.3e\n", info.iters, k,
                    fp32 ? "fp32" : "fp64", theta, rn);

        if (fp32) {
            // The FP32 phase ends at fp32_switch_resid, or when the residual
            // has stopped improving close to the FP32 rounding floor of the
            // sigma build (taken as 2e-6 |theta|); a plateau well above that
            // floor is slow convergence, which FP64 would not cure.
            if (rn < 0.98 * best_rn) {
                best_rn = rn;
                since_best = 0;
            } else {
                ++since_best;
            }
            const bool at_floor = rn < 10.0 * 2e-6 * std::fabs(theta);
            if (rn <= o.fp32_switch_resid || (since_best >= 20 && at_floor) || force_fp64 ||
                info.iters >= o.max_iter / 2) {
                // correction phase: restart from the Ritz vector with FP64 sigma builds
                fp32 = false;
                TB_HIP(hipMemcpyAsync(V[0], X, n * sizeof(double), hipMemcpyDeviceToDevice, st));
                sigma(V[0], W[0]);
                multidot(V, 1, W[0], col.data());
                G[0] = col[0];
                k = 1;
                theta = col[0];
                yprev.clear();
                continue;
            }
        } else if (rn <= o.tol_resid &&
                   (o.tol_energy <= 0.0 || std::fabs(theta - theta_prev) <= o.tol_energy)) {
            converged = true;
            break;
        }
        if (info.iters >= o.max_iter) break;
        if (abort && abort->load()) {
            info.energy = theta;
            info.resid_norm = rn;
            info.converged = 0;
            return TBSCI_E_STATE;
        }
        if (k >= nmax) {
            // restart: keep the Ritz vector x = V y and the part of the
            // previous Ritz vector orthogonal to it, z = yp - (yp.y) y
            std::vector<double> z(k);
            double dz = 0.0, nz = 0.0;
            for (int i = 0; i < k; ++i) dz += yp[i] * y[i];
            for (int i = 0; i < k; ++i) {
                z[i] = yp[i] - dz * y[i];
                nz += z[i] * z[i];
            }
            nz = std::sqrt(nz);
            std::swap(V[0], X);
            std::swap(W[0], WX);
            bool two = false;
            if (nz > 1e-8 && nmax >= 3) {  // room for x, the previous direction and t
                for (int i = 0; i < k; ++i) z[i] /= nz;
                TB_HIP(hipMemcpyAsync(ydev, z.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
                // X / WX now hold the old V[0] / W[0]: V and W of the old basis
                // are read through a list that maps slot 0 to them
                std::vector<double *> Vo(V.begin(), V.begin() + k), Wo(W.begin(), W.begin() + k);
                Vo[0] = X;
                Wo[0] = WX;
                k_lincomb2<<<1024, kB, 0, st>>>(n, vl(Vo, k), vl(Wo, k), k, ydev, XP, WXP);
                TB_HIP(hipGetLastError());
                TB_HIP(hipStreamSynchronize(st));  // z lives on the host stack
                // z is a difference of nearly equal vectors near convergence, so
                // V z is re-orthogonalised against x on the device (twice), with
                // the same combination applied to its image
                std::vector<double *> v0{V[0]}, w0{W[0]}, xp{XP};
                for (int pass = 0; pass < 2; ++pass) {
                    multidot(v0, 1, XP, nullptr);
                    k_sub_proj<<<1024, kB, 0, st>>>(n, vl(v0, 1), 1, dots, XP);
                    k_sub_proj<<<1024, kB, 0, st>>>(n, vl(w0, 1), 1, dots, WXP);
                }
                double n2;
                multidot(xp, 1, XP, &n2);
                if (std::sqrt(std::max(n2, 0.0)) > 1e-8) {
                    k_scale_by_rnorm<<<1024, kB, 0, st>>>(n, dots, XP);
                    k_scale_by_rnorm<<<1024, kB, 0, st>>>(n, dots, WXP);
                    double g0[2], g1[2];
                    std::vector<double *> ws2{W[0], WXP};
                    multidot(ws2, 2, V[0], g0);  // x.Wx, x.Wxp
                    multidot(ws2, 2, XP, g1);    // xp.Wx, xp.Wxp
                    std::swap(V[1], XP);
                    std::swap(W[1], WXP);
                    G[0] = g0[0];
                    G[1] = g0[1];
                    G[nmax] = g1[0];
                    G[nmax + 1] = g1[1];
                    k = 2;
                    yprev.assign({1.0, 0.0});
                    two = true;
                }
            }
            if (!two) {
                std::vector<double *> v0{V[0]};
                multidot(v0, 1, W[0], col.data());
                G[0] = col[0];
                k = 1;
                yprev.assign({1.0});
            }
        }
        // normalise t (the drop test below is relative), then two
        // Gram-Schmidt passes against V[0..k)
        {
            std::vector<double *> tv{T};
            multidot(tv, 1, T, nullptr);
            k_scale_by_rnorm<<<1024, kB, 0, st>>>(n, dots, T);
        }
        for (int pass = 0; pass < 2; ++pass) {
            multidot(V, k, T, nullptr);
            k_sub_proj<<<1024, kB, 0, st>>>(n, vl(V, k), k, dots, T);
        }
        double tn2;
        std::vector<double *> tv{T};
        multidot(tv, 1, T, &tn2);
        if (!(std::sqrt(std::max(tn2, 0.0)) >= 1e-10)) {
            if (fp32) {  // no new direction in FP32: go to the FP64 phase
                force_fp64 = true;
                continue;
            }
            break;  // stagnation
        }
        k_scale_by_rnorm<<<1024, kB, 0, st>>>(n, dots, T);
        TB_HIP(hipMemcpyAsync(V[k], T, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        sigma(V[k], W[k]);
        multidot(V, k + 1, W[k], col.data());
        for (int i = 0; i <= k; ++i) G[i * nmax + k] = G[k * nmax + i] = col[i];
        ++k;
    }
    // FP32 phase never handed over (max_iter hit): the energy is not FP64-certified
    if (fp32) converged = false;

    if (C_out) {
        k_absmax<<<gb, kB, 0, st>>>(n, X, partial, pidx);
        std::vector<double> pv(gb), xs(1);
        std::vector<int64_t> pi(gb);
        TB_HIP(hipMemcpyAsync(pv.data(), partial, gb * sizeof(double), hipMemcpyDeviceToHost, st));
        TB_HIP(hipMemcpyAsync(pi.data(), pidx, gb * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        TB_HIP(hipStreamSynchronize(st));
        double best = -1.0;
        int64_t at = 0;
        for (unsigned b = 0; b < gb; ++b)
            if (pi[b] >= 0 && (pv[b] > best || (pv[b] == best && pi[b] < at))) {
                best = pv[b];
                at = pi[b];
            }
        TB_HIP(hipMemcpyAsync(xs.data(), X + at, sizeof(double), hipMemcpyDeviceToHost, st));
        TB_HIP(hipStreamSynchronize(st));
        TB_HIP(hipMemcpyAsync(C_out, X, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        if (xs[0] < 0) k_scale_const<<<1024, kB, 0, st>>>(n, -1.0, C_out);
        TB_HIP(hipStreamSynchronize(st));
    }
    info.energy = theta;
    info.resid_norm = rn;
    info.converged = converged ? 1 : 0;
    info.t_sigma_s = t_sigma;
    info.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return converged ? TBSCI_OK : TBSCI_E_NOTCONV;
}

void check_opts(const tbsci_davidson_opts &o) {
    if (o.n_max < 2 || o.n_max > kMaxVec) throw Error(TBSCI_E_INVAL, "n_max must be in [2, 64]");
    if (o.max_iter < 1) throw Error(TBSCI_E_INVAL, "max_iter must be >= 1");
    if (o.precision != TBSCI_FP64 && o.precision != TBSCI_MIXED)
        throw Error(TBSCI_E_INVAL, "precision must be TBSCI_FP64 or TBSCI_MIXED");
    if (!(o.tol_resid > 0.0) || !(o.precond_floor > 0.0) || o.tol_energy < 0.0 ||
        !(o.fp32_switch_resid > 0.0))
        throw Error(TBSCI_E_INVAL, "tolerances must be positive");
}

}  // namespace tbsci

using namespace tbsci;

extern "C" {

void tbsci_davidson_default_opts(tbsci_davidson_opts *o) {
    if (!o) return;
    o->n_max = 8;
    o->max_iter = 200;
    o->precision = TBSCI_FP64;
    o->tol_resid = 1e-6;
    o->tol_energy = 0.0;
    o->fp32_switch_resid = 1e-4;
    o->precond_floor = 1e-8;
}

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
        if (guess_dev) check_dev(guess_dev, c->device, "guess");
        if (C_out_dev) check_dev(C_out_dev, c->device, "C_out");
        tbsci_davidson_info tmp;
        const int rc = davidson_run(*c, o, guess_dev, C_out_dev, tmp, (hipStream_t)stream);
        *info = tmp;
        if (rc == TBSCI_E_NOTCONV) set_error(rc, "Davidson did not reach the tolerance");
        return rc;
    });
}

}  // extern "C"
