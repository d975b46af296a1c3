// Internal declarations of the TPB sigma library: context layout, packed
// list entries and the kernel launchers shared by the host-side sources.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstring>
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
    // the same rows grouped by source chunk of `chunk` strings (see
    // sweep_chunk), when there is more than one chunk:
    // row I's entries with col in chunk c are b_*[a_ptr[I] + b_off[I (nch + 1) + c] ...]
    int64_t chunk = 0;
    int nch = 1;
    int32_t *b_off = nullptr;
    int32_t *b_col = nullptr;
    double *b_val = nullptr;
    float *b_val32 = nullptr;
    double *dsame = nullptr;   // [l] diagonal of the same-spin operator
    double *jocc = nullptr;    // [l][M]: sum_{r in I} (pp|rr) for each p
    int64_t n_s = 0, n_d = 0, n_a = 0;
    int max_s = 0;             // longest singles row
    // the singles rows regrouped by (16-pair MFMA tile t, lane group g) of
    // their folded pair index (same row pointers as s_ptr);
    // g_off[row * (4 ntile + 1) + 4 t + g] is the start of that group in the row
    Ent *g_ent = nullptr;
    int32_t *g_off = nullptr;
    // the strings in classes by the k-steps of their singles lists,
    // ceil(len / 4) <= 8, 16, 24, 28, 32: class k holds ks_rows[ks_off[k] ..
    // ks_off[k+1]) (the global-fragment opposite-spin kernel's launches)
    int32_t *ks_rows = nullptr;
    int64_t ks_off[6] = {0, 0, 0, 0, 0, 0};
    // hole-pair form of the same-spin operator (built on request, n >= 2):
    // the (n-2)-electron hole strings K of the spin's strings, each with
    // its entries (string x, occupied pair p<q with K = x - {p, q}, sign);
    // h_inv lists the entries of each string
    bool hole_built = false;     // hole_build ran (index on the device or not)
    bool hole = false;           // index on the device
    bool hole_auto = false;      // the automatic method takes it (see hole_build)
    int hmax = 0;                // longest hole-string list
    int npo = 0;                 // occupied pairs per string, n(n-1)/2
    int pp = 0;                  // orbital pairs p<q, M(M-1)/2
    int64_t n_hole = 0, n_hent = 0;
    double hole_mfma = 0.0;      // sum over K of its padded product block, 16 MT x 4 k-steps
    int64_t *h_ptr = nullptr;    // [n_hole + 1]
    uint2 *h_ent = nullptr;      // [n_hent]: .x string, .y pair | sign << 16
    int32_t *h_inv = nullptr;    // [l][npo] entry positions
    double *hW = nullptr;        // [pp][pp] pair-pair operator (see hole_sweep.hip)
    float *hW32 = nullptr;
};

// The beta sweep runs on C^T: for a block of alpha rows it transposes the
// block, sweeps the transposed rows with A_beta and adds the transposed
// result back into sigma.  Its workspace holds C^T and the sweep result of
// one block, 2 l_beta rows FP64 elements; blocks take every row when that
// fits in `cap` bytes, else the most rows that fit, rounded down to whole
// column tiles of the sweep on every XCD (multiples of 2048, or of 256 for
// short blocks).  0 when not even one row fits.
constexpr size_t kWorkCap = size_t(2) << 30;
inline int64_t beta_block_rows(int64_t la, int64_t lb, size_t cap) {
    const size_t per_row = 2 * (size_t)lb * sizeof(double);
    const int64_t fit = (int64_t)(cap / per_row);
    if (fit >= la) return la;
    if (fit >= 2048) return fit / 2048 * 2048;
    if (fit >= 256) return fit / 256 * 256;
    return fit;
}
inline size_t sigma_work_bytes(int64_t la, int64_t lb) {
    return 2 * (size_t)lb * (size_t)beta_block_rows(la, lb, kWorkCap) * sizeof(double);
}

// Sweep source chunk: the gathered rows of one chunk, 128 columns wide in
// FP64, fill 3 MB of an XCD's 4 MB L2
constexpr int64_t kSweepChunk = 3072;
// Panel sweep: source rows staged in LDS this many at a time
constexpr int64_t kPanelRows = 64;

// Source chunk of a spin's same-spin rows for the sweeps: kPanelRows (LDS
// panels) when the spin has at most kSweepChunk strings and its rows hold
// at least 4 entries per panel on average; kSweepChunk (one L2-resident
// pass per chunk) for more strings; 0 for a single plain pass.
inline int64_t sweep_chunk(int64_t l, int64_t n_a) {
    if (l > kSweepChunk) return kSweepChunk;
    const int64_t npc = (l + kPanelRows - 1) / kPanelRows;
    if (npc > 1 && n_a >= 4 * npc * l) return kPanelRows;
    return 0;
}

// A TBSCI space (determinant-level pruning, Sec. II.A): alpha row w keeps
// the beta strings idx[off[w] .. off[w+1]) (caller indices, ascending).
// Vectors at the boundary are compact, the kept determinants row by row;
// inside, sigma runs on the zero-extended [l_alpha][l_beta] layout and
// reads the kept entries back (the projector onto the space is diagonal in
// the TPB basis, so this is exact), and the solver keeps its vectors in that
// layout with every entry outside the space zero.
struct Dets {
    int64_t n = 0;              // kept determinants
    int64_t *off = nullptr;     // [l_alpha + 1]
    int32_t *idx = nullptr;     // [n]
    uint32_t *mask = nullptr;   // [l_alpha][wpr]: bit u of row w set when (w, u) is kept
    int64_t wpr = 0;            // 32-bit words per mask row
    bool symmetric = false;     // (w, u) kept exactly when (u, w) is kept
    bool open_pairs = false;    // some (w, u) with w != u is kept
    void *work = nullptr;       // two zero-extended vectors for the compact sigma
    size_t work_bytes = 0;
};

struct Ctx {
    int M = 0, P = 0, device = 0;
    bool flip_lists = false;    // the alpha and beta lists are identical (see flip)
    Dets *dets = nullptr;       // TBSCI space, or nullptr for the whole TPB space
    std::vector<int32_t> irreps; // orbital irreps once a symmetry is set (else empty)
    int target_irrep = -1;
    // deterministic sigma (tbsci_set_deterministic): the opposite-spin row
    // accumulates in fixed point, the sweeps run in one fixed order;
    // det_buf[0] = max |C| bits, det_buf[1] = the fixed-point scale
    bool det = false;
    double maxV = 0.0;           // largest |(pq|rs)|
    double *det_buf = nullptr;
    // rows longer than LDS: the rest of each row in fixed point, left zeroed
    // by every sigma (det_stage_n entries)
    unsigned long long *det_stage = nullptr;
    int64_t det_stage_n = 0;
    // alpha and beta lists are the same strings in the same order with
    // N_alpha = N_beta: H commutes with the spin flip C -> C^T (up to the
    // sign (-1)^N), and the solvers work in the C^T = C and C^T = -C
    // sectors separately
    bool flip = false;
    double *h = nullptr;     // [M][M]
    double *eri = nullptr;   // [M^4]
    double *V64 = nullptr;   // folded [P][P]: V[pair(p,q)][pair(r,s)] = (pq|rs)
    float *V32 = nullptr;
    Spin sp[2];
    // sigma workspace of the beta sweep (allocated on first use; see
    // beta_block_rows)
    void *work = nullptr;
    size_t work_bytes = 0;
    // same-spin method (tbsci_set_same_spin) and the hole-pair sweep's
    // product buffer (allocated on first use)
    int same_spin = TBSCI_SAME_SPIN_AUTO;
    void *hole_work = nullptr;
    size_t hole_work_bytes = 0;
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

// Descriptor tables of grouped launches: an append-only region of pinned
// host memory mirrored in device memory.  put() copies a table into the
// host region and enqueues its transfer on the stream; the tables of one
// round of launches stay valid until reset(), which the owner calls only
// after the stream has drained.
struct TableArena {
    unsigned char *host = nullptr, *dev = nullptr;
    size_t cap = 0, off = 0;
    explicit TableArena(size_t bytes) : cap(bytes) {
        TB_HIP(hipHostMalloc((void **)&host, cap, hipHostMallocDefault));
        if (hipMalloc((void **)&dev, cap) != hipSuccess) {
            (void)hipHostFree(host);
            host = nullptr;
            throw Error(TBSCI_E_NOMEM, "descriptor table allocation failed");
        }
    }
    ~TableArena() {
        if (dev) (void)hipFree(dev);
        if (host) (void)hipHostFree(host);
    }
    TableArena(const TableArena &) = delete;
    TableArena &operator=(const TableArena &) = delete;
    // copy a table into the host region; its device copy is made by flush()
    template <typename D>
    const D *stage(const D *src, size_t n) {
        const size_t bytes = n * sizeof(D), at = off;
        if (bytes == 0) return nullptr;
        if (at + bytes > cap) throw Error(TBSCI_E_NOMEM, "descriptor tables exceed their arena");
        memcpy(host + at, src, bytes);
        off = (at + bytes + 255) & ~size_t(255);
        return (const D *)(dev + at);
    }
    // enqueue one transfer of everything staged since the last flush
    void flush(hipStream_t st) {
        if (off > flushed)
            TB_HIP(hipMemcpyAsync(dev + flushed, host + flushed, off - flushed,
                                  hipMemcpyHostToDevice, st));
        flushed = off;
    }
    void reset() { off = flushed = 0; }
    size_t flushed = 0;
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

// ---- api.hip
// validation of a problem (throws TBSCI_E_INVAL with a message)
void validate_problem(int M, int n_alpha, int n_beta, const double *h, const double *eri,
                      const uint64_t *alpha, int64_t l_alpha, const uint64_t *beta,
                      int64_t l_beta);
void check_device_index(int device);
// a context of validated inputs (synchronous; throws on device errors)
Ctx *create_ctx(int M, int n_alpha, int n_beta, const double *h, const double *eri,
                const uint64_t *alpha, int64_t l_alpha, const uint64_t *beta, int64_t l_beta,
                int device);
void destroy_ctx(Ctx *c);
// device bytes a context holds (page-rounded allocation sizes, sigma
// workspace included), and an upper bound of it, transients of the list
// build included, from the problem shape alone
size_t ctx_bytes(const Ctx &c);
size_t ctx_bytes_bound(int M, int n_alpha, int n_beta, int64_t l_alpha, int64_t l_beta);

Ctx *ctx_of(const tbsci_ctx *p);
// sigma on the context's space (the TPB space, or its TBSCI space with
// compact vectors); terms as tbsci_sigma_terms
void sigma_any(Ctx &c, const void *C, void *S, int precision, hipStream_t st, int terms);
void check_ctx(const tbsci_ctx *ctx);
void check_dev(const void *p, int device, const char *name);

// ---- dets.hip (TBSCI spaces)
void free_dets(Ctx &c);
// compact (dets->n entries) -> zero-extended [l_alpha][l_beta] of the same
// type (sz = 8 or 4 bytes), and back
void dets_expand(Ctx &c, const void *compact, void *dense, size_t sz, hipStream_t st);
void dets_gather(Ctx &c, const void *dense, void *compact, size_t sz, hipStream_t st);
// zero the entries of a zero-extended FP64 vector that are not kept
void dets_mask(Ctx &c, double *dense, hipStream_t st);
// the two zero-extended FP64 vectors of the compact sigma (allocated on first use)
double *dets_work(Ctx &c);
// validate a layout and make it the context's space (throws TBSCI_E_INVAL)
void install_dets(Ctx &c, const int64_t *row_off, const int32_t *beta_idx);

// ---- launchers (index_kernels.hip)
void build_spin(Ctx &c, Spin &s, const uint64_t *host_str, hipStream_t st);
void launch_lookup(const Spin &s, const uint64_t *q, int64_t n, int32_t *out, hipStream_t st);
// drop the same-spin elements that are exactly zero (the diagonal stays
// first in each row) and rebuild the source-chunked copy; synchronous
void compact_same_spin(Ctx &c, Spin &s, hipStream_t st);
void launch_full_diag(const Ctx &c, double *out, hipStream_t st);

// ---- launchers (sigma_kernels.hip)
// sigma with the context's workspace (allocated on first use)
void launch_sigma(Ctx &c, const void *C, void *S, int precision, hipStream_t st, int terms = 7);
// sigma with a caller-provided workspace of work_bytes bytes (the beta
// sweep runs in blocks that fit; throws TBSCI_E_INVAL when one row does
// not); marks: record the measurement events when timing is on (they are
// created on first use, an allocation)
// fixed-point staging entries deterministic sigma needs for this context
int64_t det_stage_entries(const Ctx &c);
// hole-pair sweep (hole_sweep.hip): build a spin's hole-string index and
// pair operator; whether a spin's same-spin term takes it; its product
// buffer; Y = A_s X for a spin (X, Y: [l_s][ncols], precision's type)
void hole_build(Ctx &c, int spin, bool force);
bool hole_on(const Ctx &c, int spin);
bool hole_any(const Ctx &c);
void *hole_workspace(Ctx &c);
void hole_sweep(Ctx &c, int spin, int64_t ncols, const void *X, void *Y, int precision,
                void *work, size_t work_bytes, hipStream_t st);
void free_hole(Spin &s);
// build a spin's k-step classes (ks_rows, ks_off) from its singles lists
void build_ks_classes(Spin &s);
void launch_sigma_ws(Ctx &c, const void *C, void *S, int precision, hipStream_t st, int terms,
                     void *work, size_t work_bytes, bool marks, void *hwork = nullptr,
                     size_t hbytes = 0);
double executed_flops(Ctx &c, int kernel, int precision);
// sigma of n problems in shared launches (one per kernel type, the
// opposite-spin term one per group of equal tile shape); C[i], S[i] are
// device arrays of precision `precision` for ctx[i].  Tables go to `ar`.
void launch_sigma_group(Ctx *const *ctx, const void *const *C, void *const *S, int n,
                        int precision, TableArena &ar, hipStream_t st);
// make sure the sigma workspace of c exists (allocates)
void reserve_sigma_workspace(Ctx &c);

// ---- davidson.hip
// T = (T + tau T^T) / 2 in place for a square l x l row-major matrix
// (tau = +1 or -1), one 256-thread block per 32 x 32 tile pair (bi <= bj;
// blocks with bi > bj return); used on correction vectors to keep a
// flip-symmetric solve in the C^T = tau C sector
__device__ __forceinline__ void flip_sym_block(int64_t b, int64_t l, double tau,
                                               double *__restrict__ T) {
    __shared__ double A[32][33], B[32][33];
    const int64_t nt = (l + 31) / 32, bi = b / nt, bj = b - bi * nt;
    if (bi > bj) return;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = bi * 32 + r, j = bj * 32 + tx;
        A[r][tx] = (i < l && j < l) ? T[i * l + j] : 0.0;
        const int64_t i2 = bj * 32 + r, j2 = bi * 32 + tx;
        B[r][tx] = (i2 < l && j2 < l) ? T[i2 * l + j2] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = bi * 32 + r, j = bj * 32 + tx;
        if (i < l && j < l) T[i * l + j] = 0.5 * (A[r][tx] + tau * B[tx][r]);
        const int64_t i2 = bj * 32 + r, j2 = bi * 32 + tx;
        if (i2 < l && j2 < l) T[i2 * l + j2] = 0.5 * (B[r][tx] + tau * A[tx][r]);
    }
}

void check_opts(const tbsci_davidson_opts &o);

}  // namespace tbsci
