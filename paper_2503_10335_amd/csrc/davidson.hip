// Host-side pieces of the Davidson solver (paper Sec. II.B): the k x k
// projected eigenproblem, option checks and defaults.  The iteration itself
// runs in the solver engine (batch.hip) on the device.
#include <cmath>
#include <vector>

#include "batch.hpp"

namespace tbsci {

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

void check_opts(const tbsci_davidson_opts &o) {
    if (o.n_max < 2 || o.n_max > kBatchMaxVec)
        throw Error(TBSCI_E_INVAL, "n_max must be in [2, 16]");
    if (o.max_iter < 1) throw Error(TBSCI_E_INVAL, "max_iter must be >= 1");
    if (o.precision != TBSCI_FP64 && o.precision != TBSCI_MIXED)
        throw Error(TBSCI_E_INVAL, "precision must be TBSCI_FP64 or TBSCI_MIXED");
    if (!(o.tol_resid > 0.0) || !(o.precond_floor > 0.0) || o.tol_energy < 0.0 ||
        !(o.fp32_switch_resid > 0.0))
        throw Error(TBSCI_E_INVAL, "tolerances must be positive");
    if (o.guess_kind != TBSCI_GUESS_DIAG && o.guess_kind != TBSCI_GUESS_USER &&
        o.guess_kind != TBSCI_GUESS_SUBSPACE)
        throw Error(TBSCI_E_INVAL, "guess_kind must be TBSCI_GUESS_DIAG, _USER or _SUBSPACE");
    if (o.guess_strings < 0) throw Error(TBSCI_E_INVAL, "guess_strings must be >= 0");
    if (o.sector < -1 || o.sector > 1) throw Error(TBSCI_E_INVAL, "sector must be -1, 0 or 1");
    if (o.storage != TBSCI_STORE_AUTO && o.storage != TBSCI_STORE_FULL &&
        o.storage != TBSCI_STORE_LEAN)
        throw Error(TBSCI_E_INVAL, "storage must be TBSCI_STORE_AUTO, _FULL or _LEAN");
}

}  // namespace tbsci

using namespace tbsci;

extern "C" {

void tbsci_davidson_default_opts(tbsci_davidson_opts *o) {
    if (!o) return;
    o->n_max = 8;
    o->max_iter = 200;
    o->precision = TBSCI_FP64;
    o->guess_kind = TBSCI_GUESS_DIAG;
    o->sector = 0;
    o->storage = TBSCI_STORE_AUTO;
    o->guess_strings = 0;
    o->tol_resid = 1e-6;
    o->tol_energy = 0.0;
    o->fp32_switch_resid = 1e-4;
    o->precond_floor = 1e-8;
}

}  // extern "C"
