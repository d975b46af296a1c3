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
#include "tbsci_internal.hpp"

namespace tbsci {
namespace {

constexpr int kBlock = 256;

template <typename T>
struct Vals;
template <>
struct Vals<double> {
    static const double *a(const Spin &s) { return s.a_val; }
    static const double *V(const Ctx &c) { return c.V64; }
};
template <>
struct Vals<float> {
    static const float *a(const Spin &s) { return s.a_val32; }
    static const float *V(const Ctx &c) { return c.V32; }
};

// alpha-alpha row sweep: sigma[I, :] = sum_J A_a[I, J] C[J, :] (overwrites).
// One block per (row I, column block); list entries are block-uniform, the
// C rows are read coalesced.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_aa_sweep(int64_t lb, int64_t ncb,
                                                     const int64_t *__restrict__ a_ptr,
                                                     const int32_t *__restrict__ a_col,
                                                     const T *__restrict__ a_val,
                                                     const T *__restrict__ C, T *__restrict__ S) {
    const int64_t I = blockIdx.x / ncb;
    const int64_t col = (blockIdx.x - I * ncb) * kBlock + threadIdx.x;
    if (col >= lb) return;
    T acc = 0;
    const int64_t e1 = a_ptr[I + 1];
    for (int64_t e = a_ptr[I]; e < e1; ++e) acc += a_val[e] * C[(int64_t)a_col[e] * lb + col];
    S[I * lb + col] = acc;
}

// beta-beta column sweep: sigma[I, I'] += sum_J' A_b[I', J'] C[I, J'].
// Thread per column I', R alpha rows per block so each list entry is reused.
template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_bb_sweep(int64_t la, int64_t lb, int64_t ncb,
                                                     const int64_t *__restrict__ b_ptr,
                                                     const int32_t *__restrict__ b_col,
                                                     const T *__restrict__ b_val,
                                                     const T *__restrict__ C, T *__restrict__ S) {
    const int64_t rb = blockIdx.x / ncb;
    const int64_t Ip = (blockIdx.x - rb * ncb) * kBlock + threadIdx.x;
    if (Ip >= lb) return;
    const int64_t I0 = rb * R;
    T acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0;
    const int64_t e1 = b_ptr[Ip + 1];
    for (int64_t e = b_ptr[Ip]; e < e1; ++e) {
        const int64_t j = b_col[e];
        const T v = b_val[e];
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (I0 + r < la) acc[r] += v * C[(I0 + r) * lb + j];
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (I0 + r < la) S[(I0 + r) * lb + Ip] += acc[r];
}

// Opposite-spin term, direct double sum:
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

template <typename T>
void sigma_impl(Ctx &c, const T *C, T *S, hipStream_t st) {
    const Spin &A = c.sp[0], &B = c.sp[1];
    const int64_t la = A.l, lb = B.l;
    const int64_t ncb = (lb + kBlock - 1) / kBlock;
    k_aa_sweep<T><<<(unsigned)(la * ncb), kBlock, 0, st>>>(lb, ncb, A.a_ptr, A.a_col, Vals<T>::a(A),
                                                            C, S);
    TB_HIP(hipGetLastError());
    constexpr int R = 8;
    const int64_t nrb = (la + R - 1) / R;
    k_bb_sweep<T, R><<<(unsigned)(nrb * ncb), kBlock, 0, st>>>(la, lb, ncb, B.a_ptr, B.a_col,
                                                                 Vals<T>::a(B), C, S);
    TB_HIP(hipGetLastError());
    k_ab_direct<T><<<(unsigned)(la * ncb), kBlock, 0, st>>>(lb, ncb, c.P, A.s_ptr, A.s_ent, B.s_ptr,
                                                             B.s_ent, Vals<T>::V(c), C, S);
    TB_HIP(hipGetLastError());
}

}  // namespace

void launch_sigma(Ctx &c, const void *C, void *S, int precision, hipStream_t st) {
    if (precision == TBSCI_FP64)
        sigma_impl<double>(c, (const double *)C, (double *)S, st);
    else
        sigma_impl<float>(c, (const float *)C, (float *)S, st);
}

}  // namespace tbsci
