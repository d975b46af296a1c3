// Point-group symmetry (paper Sec. II.A: only the symmetry-allowed
// determinants of the TPB space are kept, and with the beta strings sorted
// by irrep each I_w is one contiguous interval; Sec. II.D: two alpha strings
// of different irreps differing by two orbitals have vanishing same-spin
// elements, so their pairs are skipped).
//
// Irreps of the abelian point groups (D2h and its subgroups) are integer
// labels 0..7 whose product is their XOR.  A string's irrep is the product
// of its occupied orbitals' irreps; a determinant's is the product of its two
// strings'.  tbsci_set_symmetry keeps the determinants of one total irrep
// (a TBSCI space, dets.hip) and drops from the same-spin operators the
// elements that are exactly zero by symmetry, so the sweeps skip them.
#include <algorithm>
#include <cmath>

#include "tbsci_internal.hpp"

namespace tbsci {
namespace {

struct IrrepTable {
    int8_t g[64];
};

// out[i] = XOR of the irreps of the orbitals occupied in str[i]
__global__ __launch_bounds__(256) void k_string_irrep(const uint64_t *__restrict__ str, int64_t l,
                                                      IrrepTable t, int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= l) return;
    int g = 0;
    for (uint64_t m = str[i]; m; m &= m - 1) g ^= t.g[__builtin_ctzll(m)];
    out[i] = g;
}

std::vector<int32_t> string_irreps(const Ctx &c, int spin, hipStream_t st) {
    const Spin &s = c.sp[spin];
    IrrepTable t{};
    for (int p = 0; p < c.M; ++p) t.g[p] = (int8_t)c.irreps[p];
    int32_t *d = nullptr;
    TB_HIP(hipMalloc((void **)&d, sizeof(int32_t) * std::max<int64_t>(s.l, 1)));
    std::vector<int32_t> h((size_t)s.l);
    try {
        k_string_irrep<<<(unsigned)((s.l + 255) / 256), 256, 0, st>>>(s.str, s.l, t, d);
        TB_HIP(hipGetLastError());
        TB_HIP(hipMemcpyAsync(h.data(), d, sizeof(int32_t) * s.l, hipMemcpyDeviceToHost, st));
        TB_HIP(hipStreamSynchronize(st));
    } catch (...) {
        (void)hipFree(d);
        throw;
    }
    TB_HIP(hipFree(d));
    return h;
}

// the integrals must be totally symmetric in the irreps (to 1e-12 of their
// largest magnitude), else the kept determinants would not decouple
void check_symmetric_integrals(const Ctx &c, const int32_t *irr) {
    const int M = c.M;
    const size_t M2 = (size_t)M * M, M4 = M2 * M2;
    std::vector<double> h(M2), eri(M4);
    TB_HIP(hipMemcpy(h.data(), c.h, sizeof(double) * M2, hipMemcpyDeviceToHost));
    TB_HIP(hipMemcpy(eri.data(), c.eri, sizeof(double) * M4, hipMemcpyDeviceToHost));
    double hm = 0.0, em = 0.0;
    for (double v : h) hm = std::max(hm, std::fabs(v));
    for (double v : eri) em = std::max(em, std::fabs(v));
    for (int p = 0; p < M; ++p)
        for (int q = 0; q < M; ++q)
            if (irr[p] != irr[q] && std::fabs(h[(size_t)p * M + q]) > 1e-12 * hm)
                throw Error(TBSCI_E_INVAL, "h couples orbitals of different irreps");
    for (int p = 0; p < M; ++p)
        for (int q = 0; q < M; ++q)
            for (int r = 0; r < M; ++r)
                for (int s = 0; s < M; ++s)
                    if ((irr[p] ^ irr[q] ^ irr[r] ^ irr[s]) != 0 &&
                        std::fabs(eri[(((size_t)p * M + q) * M + r) * M + s]) > 1e-12 * em)
                        throw Error(TBSCI_E_INVAL, "(pq|rs) is not totally symmetric in the "
                                                   "given irreps");
}

}  // namespace
}  // namespace tbsci

using namespace tbsci;

extern "C" {

int tbsci_set_symmetry(tbsci_ctx *ctx, const int32_t *orb_irrep, int32_t target_irrep) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        Ctx *c = ctx_of(ctx);
        if (!orb_irrep) throw Error(TBSCI_E_INVAL, "orb_irrep is NULL");
        for (int p = 0; p < c->M; ++p)
            if (orb_irrep[p] < 0 || orb_irrep[p] > 7)
                throw Error(TBSCI_E_INVAL, "orbital irreps must be labels 0..7");
        if (target_irrep < 0 || target_irrep > 7)
            throw Error(TBSCI_E_INVAL, "target_irrep must be a label 0..7");
        check_symmetric_integrals(*c, orb_irrep);
        std::vector<int32_t> keep_irr = c->irreps;
        c->irreps.assign(orb_irrep, orb_irrep + c->M);
        hipStream_t st = nullptr;
        try {
            const std::vector<int32_t> ga = string_irreps(*c, 0, st), gb = string_irreps(*c, 1, st);
            // beta strings of each irrep, ascending; with irrep-sorted beta
            // strings each list is one interval
            std::vector<int32_t> by[8];
            for (int64_t u = 0; u < c->sp[1].l; ++u) by[gb[(size_t)u]].push_back((int32_t)u);
            const int64_t la = c->sp[0].l;
            std::vector<int64_t> off((size_t)la + 1, 0);
            for (int64_t w = 0; w < la; ++w)
                off[(size_t)w + 1] = off[(size_t)w] + (int64_t)by[ga[(size_t)w] ^ target_irrep].size();
            if (off[(size_t)la] < 1)
                throw Error(TBSCI_E_INVAL, "no determinant of the target irrep");
            std::vector<int32_t> idx((size_t)off[(size_t)la]);
            for (int64_t w = 0; w < la; ++w) {
                const auto &v = by[ga[(size_t)w] ^ target_irrep];
                std::copy(v.begin(), v.end(), idx.begin() + off[(size_t)w]);
            }
            install_dets(*c, off.data(), idx.data());
        } catch (...) {
            c->irreps = keep_irr;
            throw;
        }
        c->target_irrep = target_irrep;
        // same-spin elements between strings of different irreps are exact
        // zeros with symmetric integrals: drop them from the sweeps
        for (Spin &s : c->sp) compact_same_spin(*c, s, st);
        return TBSCI_OK;
    });
}

int tbsci_string_irreps(const tbsci_ctx *ctx, int spin, int32_t *out_host) {
    return guarded([&]() -> int {
        check_ctx(ctx);
        const Ctx *c = ctx_of(ctx);
        if (spin != 0 && spin != 1) throw Error(TBSCI_E_INVAL, "spin must be 0 or 1");
        if (!out_host) throw Error(TBSCI_E_INVAL, "output is NULL");
        if (c->irreps.empty()) throw Error(TBSCI_E_STATE, "no symmetry has been set");
        const std::vector<int32_t> g = string_irreps(*c, spin, nullptr);
        std::copy(g.begin(), g.end(), out_host);
        return TBSCI_OK;
    });
}

}  // extern "C"
