// Internal declarations of the TPB sigma library: context layout, packed
// list entries and the kernel launchers shared by the host-side sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tbsci.h"

namespace tbsci {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define TB_HIP(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            throw ::tbsci::Error(e_ == hipErrorOutOfMemory ? TBSCI_E_NOMEM : TBSCI_E_DEVICE, \
                                 std::string(#x) + ": " + hipGetErrorString(e_));          \
    } while (0)

// Packed list entry (8 bytes).  j = caller index of the connected string.
//  singles: o = p | q<<6 | neg<<12 | pair(p,q)<<16   (pair = folded index)
//  doubles: o = i | jj<<6 | a<<12 | b<<18 | neg<<24
struct Ent {
    int32_t j;
    uint32_t o;
};

__host__ __device__ inline int fold_pair(int p, int q) {
    int hi = p > q ? p : q, lo = p > q ? q : p;
    return hi * (hi + 1) / 2 + lo;
}

// Per-spin device structures built at create time.
struct Spin {
    int n = 0;              // electrons per string
    int64_t l = 0;          // selected strings
    uint64_t *str = nullptr;   // [l] caller order
    uint64_t *keys = nullptr;  // [l] ascending
    int32_t *pos = nullptr;    // [l] caller index of keys[k]
    int64_t *s_ptr = nullptr;  // [l+1] E_pq links incl. p == q
    Ent *s_ent = nullptr;
    int64_t *d_ptr = nullptr;  // [l+1] doubles
    Ent *d_ent = nullptr;
    int64_t *a_ptr = nullptr;  // [l+1] same-spin operator, diagonal first
    int32_t *a_col = nullptr;
    double *a_val = nullptr;
    float *a_val32 = nullptr;
    double *dsame = nullptr;   // [l] diagonal of the same-spin operator
    double *jocc = nullptr;    // [l][M]: sum_{r in I} (pp|rr) for each p
    int64_t n_s = 0, n_d = 0, n_a = 0;
    int max_s = 0;             // longest singles row
    // the singles rows regrouped by (16-pair MFMA tile t, lane group g) of
    // their folded pair index (same row pointers as s_ptr);
    // g_off[row * (4 ntile + 1) + 4 t + g] is the start of that group in the row
    Ent *g_ent = nullptr;
    int32_t *g_off = nullptr;
};

struct Ctx {
    int M = 0, P = 0, device = 0;
    double *h = nullptr;     // [M][M]
    double *eri = nullptr;   // [M^4]
    double *V64 = nullptr;   // folded [P][P]: V[pair(p,q)][pair(r,s)] = (pq|rs)
    float *V32 = nullptr;
    Spin sp[2];
    // sigma workspace (grown on demand)
    void *work = nullptr;
    size_t work_bytes = 0;
    // per-kernel event timing (measurement only)
    bool timing = false;
    struct TimedCall {
        int precision;
        hipEvent_t ev[TBSCI_N_KERNELS + 1];
    };
    std::vector<TimedCall> timed;
    // kernels whose dynamic LDS limit has been raised (kernel, bytes)
    std::vector<std::pair<const void *, size_t>> lds_set;
};

// records an event on st if timing is on; index 0..TBSCI_N_KERNELS
void timing_mark(Ctx &c, int index, int precision, hipStream_t st);
void timing_clear(Ctx &c);

extern thread_local std::string g_err;

inline int set_error(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

// Run f, turning exceptions into status codes and a thread-local message.
template <class F>
int guarded(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        return set_error(e.code, e.what());
    } catch (const std::bad_alloc &) {
        return set_error(TBSCI_E_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return set_error(TBSCI_E_DEVICE, e.what());
    }
}

Ctx *ctx_of(const tbsci_ctx *p);
void check_ctx(const tbsci_ctx *ctx);
void check_dev(const void *p, int device, const char *name);

// ---- launchers (index_kernels.hip)
void build_spin(Ctx &c, Spin &s, const uint64_t *host_str, hipStream_t st);
void launch_lookup(const Spin &s, const uint64_t *q, int64_t n, int32_t *out, hipStream_t st);
void launch_full_diag(const Ctx &c, double *out, hipStream_t st);
void launch_diag_argmin(const Ctx &c, double *part_val, int64_t *part_idx, int nblk, hipStream_t st);

// ---- launchers (sigma_kernels.hip)
void launch_sigma(Ctx &c, const void *C, void *S, int precision, hipStream_t st, int terms = 7);
double executed_flops(Ctx &c, int kernel, int precision);

// ---- davidson.hip
int davidson_run(Ctx &c, const tbsci_davidson_opts &o, const double *guess, double *C_out,
                 tbsci_davidson_info &info, hipStream_t st);
void check_opts(const tbsci_davidson_opts &o);

}  // namespace tbsci
