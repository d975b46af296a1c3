/*
 * tbsci.h -- C ABI of the MI355X TPB sigma library (libtbsci.so).
 *
 * The library builds sigma = H*C over a tensor-product-bitstring (TPB)
 * determinant space and finds the lowest eigenpair with a Davidson solver,
 * all on one AMD Instinct GPU (gfx950).  Reference: arXiv 2503.10335,
 * "A Scalable Diagonalization Framework for Tensor-Product Bitstring
 * Selected Configuration Interaction".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Orbitals p = 0..M-1 are spatial orbitals; a string is a uint64 with bit
 *   p set when orbital p is occupied (M <= 64).
 * - The determinant space is every product of a selected alpha string with a
 *   selected beta string (Sec. II.A, Eq. TPB_Det).  The CI vector C and
 *   sigma are row-major matrices [l_alpha][l_beta]: the determinant index
 *   runs fastest over beta (Sec. II.A, the index map K = (w-1) l_beta + u,
 *   here 0-based K = i_alpha * l_beta + i_beta), rows and columns in the
 *   caller's list order.
 * - H = sum_{pq,s} h_pq a+_ps a_qs + 1/2 sum_{pqrs,st} (pq|rs) a+_ps a+_rt a_st a_qs
 *   with real integrals; (pq|rs) in chemists' notation.  Excitations that
 *   leave the selected space are projected out: sigma = P H P C.
 * - A determinant is the product of alpha creators (ascending orbital) and
 *   then beta creators (ascending orbital) on the vacuum.
 * - Every function returns an int status (TBSCI_OK = 0, TBSCI_PENDING = 1,
 *   errors < 0) and never aborts; tbsci_last_error() gives a message
 *   (thread-local).  On error, caller-owned outputs are left untouched.
 * - Host pointers are read during the call only; the library deep-copies
 *   what it keeps.  Device pointers are caller-owned allocations on the
 *   context's device (for example torch tensors' data_ptr()).  A stream
 *   argument is a hipStream_t owned by the caller; NULL is the default
 *   stream.  A context is not thread-safe: one caller thread at a time.
 */
#ifndef TBSCI_H
#define TBSCI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TBSCI_OK 0
#define TBSCI_PENDING 1
#define TBSCI_E_INVAL (-1)    /* invalid argument or input data            */
#define TBSCI_E_NOMEM (-2)    /* device or host allocation failed          */
#define TBSCI_E_DEVICE (-3)   /* HIP runtime error                         */
#define TBSCI_E_NOTCONV (-4)  /* Davidson hit max_iter or stagnated        */
#define TBSCI_E_NOTFOUND (-5) /* unknown ticket                            */
#define TBSCI_E_STATE (-6)    /* call not valid in the object's state      */

/* element type of C and sigma in tbsci_sigma */
#define TBSCI_FP64 0
#define TBSCI_FP32 1 /* FP32 inputs, outputs and arithmetic (MFMA and sweeps
                        accumulate in FP32); the opposite-spin scatter adds
                        into an FP64 copy of the output row where it fits in
                        LDS, rounded to FP32 once per row                    */
/* Davidson precision: FP32 sigma phase, then FP64 correction phase        */
#define TBSCI_MIXED 2

typedef struct tbsci_ctx tbsci_ctx;

/*
 * Create a context: validate the inputs, copy them to the device, build the
 * sorted string index (Sec. II.C: membership of an excited string in the
 * selected set by sorted list and binary search), the in-selection
 * excitation lists of both spins (Sec. II.C: single and double excitation
 * link tables, precomputed once and reused by every sigma), the same-spin
 * operator values and the folded (pq|rs) block.
 *
 *   M         number of spatial orbitals, 1..64
 *   n_alpha   electrons per alpha string (0..M); n_beta likewise
 *   h         host, M*M row-major, symmetric to 1e-12 relative
 *   eri       host, M^4 row-major, eri[((p*M+q)*M+r)*M+s] = (pq|rs), with the
 *             8-fold symmetry of real orbitals to 1e-12 relative
 *   alpha     host, l_alpha unique strings, each with n_alpha bits below M
 *   beta      host, l_beta unique strings, each with n_beta bits below M
 *   device    HIP device ordinal
 *   out       receives the context; untouched on error
 * Errors: TBSCI_E_INVAL for any violated condition above, l < 1,
 * l > 2^31-1 or a NULL pointer; TBSCI_E_NOMEM / TBSCI_E_DEVICE.
 */
int tbsci_create(int M, int n_alpha, int n_beta, const double *h, const double *eri,
                 const uint64_t *alpha, int64_t l_alpha, const uint64_t *beta,
                 int64_t l_beta, int device, tbsci_ctx **out);

/* Free the context and its device memory.  NULL-safe. */
void tbsci_destroy(tbsci_ctx *ctx);

/*
 * Sizes: l_alpha, l_beta and n_det = l_alpha * l_beta, or the number of kept
 * determinants of a TBSCI space (tbsci_set_dets).  Any output may be NULL.
 */
int tbsci_dims(const tbsci_ctx *ctx, int64_t *l_alpha, int64_t *l_beta, int64_t *n_det);

/*
 * Restrict the context to a TBSCI space (Sec. II.A: determinant-level
 * pruning of the TPB space; alpha string w is paired only with the beta
 * strings of its index set I_w, the CI vector is stored segment by segment
 * with per-segment offsets and lengths; Algorithm 1: an element enters sigma
 * only when both its determinants are kept).
 *
 *   row_off   host, l_alpha + 1 entries: row w's segment is
 *             [row_off[w], row_off[w+1]); row_off[0] = 0, nondecreasing,
 *             at most l_beta per row; n_det = row_off[l_alpha] >= 1
 *   beta_idx  host, n_det caller beta indices, ascending within a row
 * Both NULL: back to the whole TPB space.  Afterwards tbsci_sigma,
 * tbsci_sigma_terms, tbsci_diag and tbsci_davidson take and return compact
 * vectors of n_det elements in that order (sigma = P H P C with P the
 * projector onto the kept determinants).  The sigma kernels run on the
 * vector extended by zeros to [l_alpha][l_beta] and read the kept entries
 * back (exact, at the cost of the TPB space's work); the context holds two
 * such FP64 vectors, allocated on the first compact sigma, and the solver
 * keeps its vectors in that layout.  A space that maps onto itself under
 * (w, u) -> (u, w) keeps the spin-flip sectors of identical lists.
 * tbsci_sigma_batch and tbsci_sigma_noalloc reject TBSCI spaces.
 * TBSCI_E_INVAL for a malformed layout (the previous space stays).
 */
int tbsci_set_dets(tbsci_ctx *ctx, const int64_t *row_off, const int32_t *beta_idx);

/*
 * Copy the context's TBSCI layout (as given to tbsci_set_dets or built by
 * tbsci_set_symmetry) to host buffers of l_alpha + 1 and n_det entries.
 * TBSCI_E_STATE when the context holds the whole TPB space.
 */
int tbsci_get_dets(const tbsci_ctx *ctx, int64_t *row_off_host, int32_t *beta_idx_host);

/*
 * Point-group symmetry (Sec. II.A: only the symmetry-allowed determinants
 * of the TPB space are kept; with the beta strings sorted by irrep, each
 * I_w is one contiguous interval; Sec. II.D: alpha strings of different
 * irreps two orbitals apart have no same-spin element).  Irreps of an
 * abelian point group (D2h or a subgroup) are labels 0..7 whose product is
 * their XOR; a string's irrep is the product over its occupied orbitals.
 *
 *   orb_irrep     host, M labels
 *   target_irrep  the total irrep (alpha string's times beta string's) of
 *                 the determinants kept
 * The integrals must be totally symmetric in these irreps (h_pq = 0 across
 * irreps, (pq|rs) = 0 unless the product of the four irreps is the totally
 * symmetric one, both to 1e-12 of their largest element), else
 * TBSCI_E_INVAL.  The call installs the layout of the kept determinants as
 * tbsci_set_dets does (beta strings in the caller's order: each I_w is an
 * interval when the caller sorted them by irrep, any subset otherwise), and
 * drops the same-spin elements that are exactly zero (between strings of
 * different irreps) from the sweeps' operators, which stay exact for the
 * whole TPB space too.  Synchronous.
 */
int tbsci_set_symmetry(tbsci_ctx *ctx, const int32_t *orb_irrep, int32_t target_irrep);

/*
 * String weights of a CI vector (Sec. III.B: the weight of an alpha or beta
 * string is the sum of the squared coefficients over the determinants that
 * contain it).  C_dev: device FP64 vector of the context's space (TPB
 * [l_alpha][l_beta], or compact for a TBSCI space); w_alpha_dev /
 * w_beta_dev: device FP64 outputs of l_alpha / l_beta entries.  Fixed-order
 * reductions: the result does not depend on the launch.  Synchronous.
 */
int tbsci_string_weights(tbsci_ctx *ctx, const double *C_dev, double *w_alpha_dev,
                         double *w_beta_dev, void *stream);

/*
 * Weight-threshold selection (Sec. III.B: strings are ranked by weight and
 * kept when their weight exceeds delta times that of the Hartree-Fock
 * string).  w_dev: device weights of one spin (tbsci_string_weights);
 * ref_string: the reference string, which must be in the list and is always
 * kept.  out_host receives the kept strings, heaviest first (ties: smaller
 * string first), *n_out their number; out_host needs room for l entries of
 * that spin.  Synchronous.
 */
int tbsci_select_strings(tbsci_ctx *ctx, int spin, const double *w_dev, double delta,
                         uint64_t ref_string, uint64_t *out_host, int64_t *n_out, void *stream);

/*
 * Histogram of the coefficient magnitudes of a CI vector of the context's
 * space (Sec. III.B, the coefficient distributions of the wavefunctions):
 * counts_host[b] = number of coefficients with log10 |c| in bin b of nbins
 * equal bins over [log10_lo, log10_hi); smaller magnitudes and zeros count in
 * bin 0, larger ones in bin nbins-1.  nbins 1..4096.  Synchronous.
 */
int tbsci_coef_histogram(tbsci_ctx *ctx, const double *C_dev, double log10_lo, double log10_hi,
                         int nbins, int64_t *counts_host, void *stream);

/* Irrep of every string of one spin (spin 0 = alpha), computed on the
 * device, to a host buffer of l entries.  TBSCI_E_STATE before
 * tbsci_set_symmetry. */
int tbsci_string_irreps(const tbsci_ctx *ctx, int spin, int32_t *out_host);

/*
 * sigma = P H P C (Sec. II.B: the matrix-vector product W = H U that
 * dominates the Davidson solver; Sec. II.C and Algorithm 1: the six
 * excitation categories [2,0] [1,1] [1,0] [0,2] [0,1] [0,0]).
 *
 *   C_dev, sigma_dev  device, [l_alpha][l_beta], double (TBSCI_FP64) or
 *                     float (TBSCI_FP32); sigma is overwritten; must not alias
 *   precision         TBSCI_FP64 or TBSCI_FP32
 *   stream            hipStream_t or NULL; the call is asynchronous
 */
int tbsci_sigma(tbsci_ctx *ctx, const void *C_dev, void *sigma_dev, int precision, void *stream);

/*
 * tbsci_sigma without any allocation, for callers that cannot allocate
 * device memory (code under HIP stream capture, serving loops or
 * harnesses that forbid hipMalloc).  Same arguments, result and errors as
 * tbsci_sigma.  Its one scratch buffer -- the beta sweep's transposed block
 * of C and the block's sweep result -- is a 64 MiB static device array
 * owned by the library, one per device, held from the library's first use
 * on that device until the process ends; the beta sweep runs in blocks of
 * alpha rows that fit in it.  Every call on one device shares that array
 * and leaves its contents behind, so calls that overlap on one device (on
 * different streams or threads) race; serialise them.  Spaces whose
 * l_beta exceeds 4,194,304 strings (one alpha row does not fit) fail with
 * TBSCI_E_INVAL.  No events are recorded for tbsci_timing_*.
 */
int tbsci_sigma_noalloc(tbsci_ctx *ctx, const void *C_dev, void *sigma_dev, int precision,
                        void *stream);

/*
 * One or more of the three terms of sigma, for verification and
 * measurement: terms is a bit mask, 1 = same-spin alpha (A_a C), 2 =
 * same-spin beta (C A_b^T), 4 = opposite spin (sum (pq|rs) E^a_pq C
 * E^b_rs^T); sigma_dev is overwritten with the sum of the selected terms
 * (terms = 7 is tbsci_sigma).  Arguments as tbsci_sigma.
 */
int tbsci_sigma_terms(tbsci_ctx *ctx, const void *C_dev, void *sigma_dev, int precision,
                      int terms, void *stream);

/*
 * Reproducible sigma (the run-to-run and alone-versus-batched equality of
 * the sigma build, Sec. II.B-C, for serving): enable != 0 makes every sigma
 * of this context bitwise identical across runs and identical whether it
 * is built alone (tbsci_sigma) or inside a batch (tbsci_sigma_batch, the
 * batched Davidson).  The opposite-spin term then sums each output element
 * in 64-bit fixed point -- a power-of-two scale, taken per call from
 * max|C|, max|(pq|rs)| and the longest single-excitation lists so that no
 * partial sum can overflow -- so the order of its atomic adds no longer
 * matters.  The same-spin terms have no atomics; a space small enough to
 * share grouped launches sweeps in the grouped launches' order (alone =
 * batched), larger ones keep their panel, chunked or hole-pair sweeps.
 * Rounding: each opposite-spin contribution is rounded to a unit of
 * 2^-62 of that bound (K_alpha K_beta max|(pq|rs)| max|C|, K = longest
 * single-excitation list), about 1e-15 relative to sigma in the tested
 * spaces.  Opposite-spin rows longer than LDS
 * holds (l_beta above about 20,000 strings) keep their remainder in a
 * device staging area of l_alpha x (l_beta - that length) 8-byte entries,
 * allocated here on enable (11 GB at l_alpha = l_beta = 48,620) and left
 * zeroed by every sigma; FP32 sigma then also keeps an 8-byte row.  The
 * call allocates 16 bytes plus that area (TBSCI_E_DEVICE when it does not
 * fit); the memory is held until tbsci_destroy.  enable == 0 returns to
 * the default (FP64 atomics in the opposite-spin rows).
 */
int tbsci_set_deterministic(tbsci_ctx *ctx, int enable);

/*
 * Method of the two same-spin terms (A_alpha C and C A_beta^T; the [2,0],
 * [0,2] categories and the same-spin parts of [1,0], [0,1], [0,0] of
 * Sec. II.C):
 *   TBSCI_SAME_SPIN_CSR   sparse sweeps over the stored same-spin operator
 *                         (each output row gathers the rows of C its
 *                         singles and doubles reach)
 *   TBSCI_SAME_SPIN_HOLE  hole-pair form: for every (N-2)-electron string
 *                         K contained in the spin's strings, the rows of C
 *                         of the strings K + {q, s} times the dense block
 *                         of the pair operator
 *                         W[pr][qs] = (pq|rs) - (ps|rq)
 *                                   + (h_pq d_rs + h_rs d_pq - h_ps d_rq - h_rq d_ps) / (N - 1)
 *                         on MFMA, each string K + {p, r} reading its row
 *                         of the product back (the one-body part folded
 *                         into W; both ends run over the spin's strings
 *                         only, so the projection is exact)
 *   TBSCI_SAME_SPIN_AUTO  (the default) the hole-pair form for a spin
 *                         whose hole strings hold at least
 *                         TBSCI_HOLE_AUTO_MIN strings on average, in a
 *                         space too large for grouped launches (the beta
 *                         sweep in blocks, above 2^27 determinants) with
 *                         no point-group symmetry set; else CSR
 * A spin with fewer than 2 electrons, or with a hole string contained in
 * more than 128 of its strings, keeps the CSR sweep.  The hole-pair index
 * (built by tbsci_create for the spins the automatic method takes, else
 * here) copies the strings and integrals to the host, sorts N(N-1)/2
 * entries per string and holds about 16 B per entry on the device; the
 * hole-pair sweep also allocates a product buffer of up to 4 GiB on first
 * use.  A context on the hole-pair sweep builds its sigma alone in batched
 * calls.  tbsci_sigma_noalloc always uses CSR.  tbsci_timing_executed_flops
 * of kernels 0 and 1 reports the MFMA work of the hole-pair sweep when it
 * is on.
 */
#define TBSCI_SAME_SPIN_AUTO 0
#define TBSCI_SAME_SPIN_CSR 1
#define TBSCI_SAME_SPIN_HOLE 2
#define TBSCI_HOLE_AUTO_MIN 32
int tbsci_set_same_spin(tbsci_ctx *ctx, int method);

/*
 * Diagonal H_KK of every determinant (Sec. II.C: the [0,0] category,
 * precomputed and stored), device double [l_alpha][l_beta], asynchronous.
 */
int tbsci_diag(tbsci_ctx *ctx, double *diag_dev, void *stream);

/* Davidson start vector */
#define TBSCI_GUESS_DIAG 0 /* unit vector(s) on the smallest diagonal element          */
#define TBSCI_GUESS_USER 1 /* the caller's vector guess_dev                             */
#define TBSCI_GUESS_SUBSPACE 2 /* the ground state of the space of the guess_strings
                              strings of each spin with the smallest same-spin diagonal,
                              solved first (per spin-flip sector) and extended by zeros */
/* Davidson vector storage */
#define TBSCI_STORE_AUTO 0 /* FULL when it fits in 90% of the free device memory       */
#define TBSCI_STORE_FULL 1 /* 2 n_max + 7 FP64 vectors (restart keeps two directions)  */
#define TBSCI_STORE_LEAN 2 /* 2 n_max + 3 FP64 vectors (plain collapse restart)        */

typedef struct {
    int n_max;                /* subspace size that triggers a restart, 2..16          */
    int max_iter;             /* cap on sigma builds (both phases together, per sector)*/
    int precision;            /* TBSCI_FP64 or TBSCI_MIXED                              */
    int guess_kind;           /* TBSCI_GUESS_DIAG or TBSCI_GUESS_USER                   */
    int sector;               /* identical alpha/beta lists only: 0 = lowest state of
                                 both spin-flip sectors, +1 = C^T = C only, -1 = C^T = -C
                                 only (ignored for other spaces and for a user guess)   */
    int storage;              /* TBSCI_STORE_AUTO, _FULL or _LEAN                        */
    int guess_strings;        /* TBSCI_GUESS_SUBSPACE: strings per spin of the subspace
                                 (0: a fifth of each list, at least 50)                 */
    double tol_resid;         /* stop when the FP64 residual norm <= tol_resid          */
    double tol_energy;        /* and |E_k - E_{k-1}| <= tol_energy (0 disables)         */
    double fp32_switch_resid; /* mixed: leave the FP32 phase below this residual        */
    double precond_floor;     /* smallest |theta - H_KK| in the preconditioner           */
} tbsci_davidson_opts;

typedef struct {
    double energy;            /* lowest eigenvalue estimate (Ritz value, FP64 sigma)   */
    double resid_norm;        /* ||H x - E x||_2 of that Ritz pair                     */
    double energy_fp64_check; /* x^T H x / x^T x of the returned Ritz vector with a
                                 fresh FP64 sigma build (certifies a mixed solve)       */
    double energy_other;      /* lowest energy found in the other spin-flip sector
                                 when both were solved, else NaN                        */
    int iters;                /* sigma builds, all phases and sectors                  */
    int iters_fp32;           /* sigma builds in FP32                                  */
    int iters_fp64;           /* sigma builds in FP64 (energy checks included)         */
    int converged;            /* 1 if the tolerances were met (in every sector solved) */
    int sector;               /* +1: returned C has C^T = C, -1: C^T = -C, 0: no sector*/
    int lean;                 /* 1 if the lean vector storage was used                 */
    double t_total_s;         /* wall time of the solve                                */
    double t_sigma_s;         /* part of it spent in sigma builds                      */
} tbsci_davidson_info;

/* Defaults: n_max 8, max_iter 200, FP64, TBSCI_GUESS_DIAG, sector 0,
 * TBSCI_STORE_AUTO, guess_strings 0, tol_resid 1e-6, tol_energy 0,
 * fp32_switch_resid 1e-4, precond_floor 1e-8. */
void tbsci_davidson_default_opts(tbsci_davidson_opts *opts);

/*
 * Lowest eigenpair of P H P by Davidson iteration (Sec. II.B: Davidson
 * diagonalisation built on the sigma product; Sec. III.C: restart keeps the
 * number of stored vectors bounded).  Gram-Schmidt, the Rayleigh-Ritz
 * projection and the residual are FP64 on the device; the k x k projected
 * eigenproblem is solved on the host.  With TBSCI_MIXED the sigma builds
 * run in FP32 until the residual drops below fp32_switch_resid (or stops
 * falling), then the solver restarts from the Ritz vector with FP64 sigma
 * builds (Sec. III.A: a matrix-vector product in single precision with
 * everything else in double).  Every solve ends with one more FP64 sigma
 * build of the Ritz vector, whose Rayleigh quotient is energy_fp64_check.
 *
 * Spin-flip sectors.  When the alpha and beta lists are the same strings in
 * the same order and N_alpha = N_beta, H commutes with exchanging the two
 * strings of every determinant, and every eigenvector can be taken with a
 * symmetric (C^T = C: even total spin) or antisymmetric (C^T = -C: odd
 * spin) CI matrix.  Rounding would slowly mix the two, so each solve is
 * kept inside one sector (its corrections are (anti)symmetrised).  With
 * sector 0 both sectors are solved one after the other and the lower state
 * is returned (info.sector tells which; info.energy_other is the other
 * one); with +1 or -1 only that sector.
 *
 *   opts      host, NULL for defaults
 *   guess_dev device double [l_alpha][l_beta]: required with
 *             TBSCI_GUESS_USER (no sector is imposed then), must be NULL
 *             otherwise.  TBSCI_GUESS_SUBSPACE (whole TPB spaces only): the
 *             library first solves, in FP64 to a residual of
 *             max(tol_resid, 1e-3), the TPB space of the guess_strings
 *             strings of each spin with the smallest same-spin diagonal
 *             (the same strings for both spins when the lists are
 *             identical), once per spin-flip sector, and starts each sector
 *             from that solution extended by zeros (a P-space start;
 *             info.t_total_s includes it).  TBSCI_GUESS_DIAG: the start is the unit vector on the
 *             smallest diagonal element (first in row-major order on ties);
 *             in a flip-symmetric space, (|I J> + |J I>)/sqrt 2 for an
 *             open-shell |I J> in the symmetric sector, and
 *             (|I J> - |J I>)/sqrt 2 on the open-shell determinant with the
 *             smallest diagonal element in the antisymmetric one
 *   C_out_dev device double [l_alpha][l_beta] or NULL: receives the Ritz
 *             vector (unit norm, largest-magnitude entry positive); during a
 *             two-sector solve it also holds the first sector's vector
 *   info      host, required
 * Returns TBSCI_OK, or TBSCI_E_NOTCONV with info filled when the tolerance
 * was not met (TBSCI_E_INVAL for a zero guess, an inconsistent guess_kind
 * or an empty requested sector).  Synchronous with respect to the host,
 * with one host synchronisation per iteration (the correction and its sigma
 * are built before the host sees that iteration's residual, so a converged
 * solve has built one sigma more than it used; info.iters counts it).
 * Allocates its workspace: with TBSCI_STORE_FULL (2 n_max + 7) FP64
 * vectors -- the basis V and its images H V, the Ritz vector and its image,
 * the correction and its image, the previous Ritz direction with its image
 * (the restart keeps it next to the Ritz vector) and the diagonal H_KK
 * (Sec. II.C: computed once and stored); with TBSCI_STORE_LEAN
 * (2 n_max + 3), the paper's count (Sec. III.C): the restart collapses to
 * the Ritz vector, the image of the correction reuses a vector of the
 * collapsed basis and H_KK is recomputed from per-string parts.  MIXED adds
 * two FP32 vectors.  The sigma builds use the context's bounded workspace.
 */
int tbsci_davidson(tbsci_ctx *ctx, const tbsci_davidson_opts *opts, const double *guess_dev,
                   double *C_out_dev, tbsci_davidson_info *info, void *stream);

/*
 * Batched forms for many small problems on one device.  The work of all
 * n contexts is issued together: each kernel type of the sigma build runs
 * as one launch over every problem (the opposite-spin term one launch per
 * group of problems with the same orbital count and tile depth), and the
 * Davidson vector operations of all problems likewise, so that launch and
 * synchronisation costs are paid once per batch instead of once per
 * problem.  The arithmetic of each problem is that of the single-problem
 * call; reductions do not depend on the other members of the batch.
 *
 * tbsci_sigma_batch: sigma_dev[i] = P H P C_dev[i] for ctxs[i], i < n
 * (n <= 64, distinct contexts on one device, device arrays as in
 * tbsci_sigma, all of the given precision).  Synchronous with respect to
 * the host.
 */
int tbsci_sigma_batch(tbsci_ctx *const *ctxs, int n, const void *const *C_dev,
                      void *const *sigma_dev, int precision, void *stream);

/*
 * tbsci_davidson_batch: the lowest eigenvalue of every problem, solved in
 * lock step (one Davidson iteration of every unfinished problem per round,
 * one host synchronisation per round).  opts: NULL for defaults, else an
 * array of n (guess_kind must be TBSCI_GUESS_DIAG).  infos[i] and
 * status[i] (TBSCI_OK or TBSCI_E_NOTCONV) receive problem i's result; the
 * start vectors and sectors are those of tbsci_davidson without a guess.
 * Eigenvectors are not returned.  Each problem holds the vectors of its
 * storage mode (as tbsci_davidson) while it runs.  Returns TBSCI_OK when
 * every problem ran (whatever its own status), else an error code.
 */
int tbsci_davidson_batch(tbsci_ctx *const *ctxs, int n, const tbsci_davidson_opts *opts,
                         tbsci_davidson_info *infos, int *status, void *stream);

/* ------------------------------------------------------------------------
 * Serving: ground-state solves of many problems on one device, submitted
 * and collected asynchronously (a deployment of the Davidson solver above;
 * the paper's method is the per-request solve).
 *
 * A server owns four host threads.  Requests are admitted in arrival order
 * while their device footprint fits hbm_budget_bytes (later requests that
 * fit are admitted when the head of the queue does not); the footprint is
 * first counted as an upper bound from the problem shape and, once the
 * request's lists are built, trimmed to the bytes it holds.  Requests of
 * at most batch_ndet_threshold determinants (and n_max <= 16) run in the
 * batched solver: they join and leave between its rounds (continuous
 * batching), share its grouped sigma and vector launches, and keep their
 * Davidson subspaces in device memory until they finish.  Larger requests
 * run the single-problem solver on one of two streams of their own, at the
 * same time as the batch.  No eigenvectors are returned.
 */
typedef struct tbsci_server tbsci_server;

typedef struct {
    size_t hbm_budget;          /* bytes                                          */
    size_t hbm_reserved;        /* bytes held by admitted requests now            */
    size_t hbm_reserved_peak;   /* largest hbm_reserved so far (<= hbm_budget)    */
    int64_t submitted, completed, failed; /* failed: completed with an error     */
    int64_t queued;             /* waiting for admission                          */
    int64_t running_batched, running_solo;
    int64_t ticks;              /* rounds of the batched solver                   */
    int max_batch;              /* most requests in one round                     */
} tbsci_server_info;

/*
 * Start a server on `device`.  TBSCI_E_INVAL for a zero budget, a negative
 * threshold or a bad device.
 */
int tbsci_server_create(int device, size_t hbm_budget_bytes, int64_t batch_ndet_threshold,
                        tbsci_server **out);

/*
 * Stop: queued requests end with TBSCI_E_STATE ("cancelled"), running ones
 * are stopped at their next iteration, threads are joined and every device
 * allocation is freed.  NULL-safe.  Tickets are invalid afterwards.
 */
void tbsci_server_destroy(tbsci_server *server);

/*
 * Queue one ground-state solve.  Arguments as tbsci_create plus Davidson
 * options (NULL for defaults); every host array is copied before the call
 * returns.  Invalid inputs return TBSCI_E_INVAL and a request whose
 * footprint bound exceeds the whole budget TBSCI_E_NOMEM, both without a
 * ticket.  Thread-safe.
 */
int tbsci_submit(tbsci_server *server, int M, int n_alpha, int n_beta, const double *h,
                 const double *eri, const uint64_t *alpha, int64_t l_alpha,
                 const uint64_t *beta, int64_t l_beta, const tbsci_davidson_opts *opts,
                 uint64_t *ticket);

/*
 * State of a request: TBSCI_PENDING while queued or running; when done its
 * status (TBSCI_OK, TBSCI_E_NOTCONV, or the error that ended it, with the
 * message in tbsci_last_error) and, if out is not NULL, its result.
 * TBSCI_E_NOTFOUND for an unknown ticket.  Thread-safe; does not block.
 */
int tbsci_poll(tbsci_server *server, uint64_t ticket, tbsci_davidson_info *out);

/*
 * For a finished request: seconds from submission to admission (queue_s)
 * and to completion (latency_s), whether it ran batched, and the device
 * bytes it held.  TBSCI_PENDING while not finished, TBSCI_E_NOTFOUND for an
 * unknown ticket.  Any output pointer may be NULL.
 */
int tbsci_request_times(tbsci_server *server, uint64_t ticket, double *queue_s,
                        double *latency_s, int *batched, int64_t *footprint_bytes);

/* Counters of the server (a consistent snapshot). */
int tbsci_server_stats(tbsci_server *server, tbsci_server_info *out);

/* ------------------------------------------------------------------------
 * Inspection of the create-time structures, for verification.
 * spin: 0 = alpha, 1 = beta.
 */

/*
 * Copy the sorted string index to host buffers of l entries each:
 * keys ascending, pos[k] = caller index of keys[k] (Sec. II.C, sorted index
 * list with binary search).
 */
int tbsci_string_index(const tbsci_ctx *ctx, int spin, uint64_t *keys_host, int32_t *pos_host);

/*
 * Binary-search n query strings in the selected list of one spin on the
 * device: out_dev[i] = caller index of queries_dev[i], or -1.  Device
 * buffers, asynchronous on stream.
 */
int tbsci_lookup(const tbsci_ctx *ctx, int spin, const uint64_t *queries_dev, int64_t n,
                 int32_t *out_dev, void *stream);

/*
 * List kinds for tbsci_list_size / tbsci_get_list:
 *  1  single excitations E_pq between selected strings plus the occupation
 *     entries (p = q): row I holds (j, p, q, 0, 0, sign) with
 *     sign = <I| a+_p a_q |J_j> != 0, ordered by (p, q);
 *  2  double excitations: (j, i, jj, a, b, sign) with i < jj in I, a < b in
 *     J_j, sign = <I| a+_i a+_jj a_b a_a |J_j>, ordered by (i, jj, a, b);
 *  3  the same-spin Hamiltonian between selected strings (one-spin part of
 *     H, Sec. II.C categories [2,0] / [0,2] and the one-spin parts of
 *     [1,0] / [0,1] / [0,0]): CSR with the diagonal first in each row.
 * Rows are indexed by caller index of I.
 */
int tbsci_list_size(const tbsci_ctx *ctx, int spin, int kind, int64_t *n_entries);

/*
 * Copy a list to the host.  row_ptr_host has l+1 entries.  For kinds 1 and
 * 2, entries_host is int32 [n_entries][6]; for kind 3, entries_host is int32
 * [n_entries] column indices and values_host double [n_entries] (values_host
 * is ignored for kinds 1 and 2).
 */
int tbsci_get_list(const tbsci_ctx *ctx, int spin, int kind, int64_t *row_ptr_host,
                   int32_t *entries_host, double *values_host);

/* ------------------------------------------------------------------------
 * Measurement.  Kernels of one sigma build, by index:
 *   0  same-spin alpha sweep   (categories [2,0] and alpha parts of [1,0], [0,0])
 *   1  same-spin beta sweep    (categories [0,2] and beta parts of [0,1], [0,0])
 *   2  opposite-spin term      (category [1,1] and opposite-spin parts of
 *                               [1,0], [0,1], [0,0])
 */
#define TBSCI_N_KERNELS 3

/*
 * enable != 0: start recording HIP events around every kernel that
 * tbsci_sigma launches, on the caller's stream (previous records are
 * dropped); enable == 0: stop and drop the records.
 */
int tbsci_timing_enable(tbsci_ctx *ctx, int enable);

/*
 * For kernel index `kernel` (0..TBSCI_N_KERNELS-1) of the given precision:
 * total_ms = summed event time of its recorded launches, launches = their
 * number (waits for the recorded work to finish), flops = algorithmic
 * floating-point operations of one launch (2 per multiply-add of the
 * defining sums, not the operations the kernel executes), bytes =
 * compulsory device-memory bytes of one launch (C read once, sigma read and
 * written once, lists and values read once).  name receives a static
 * string.  Any output pointer may be NULL.
 */
int tbsci_timing_read(tbsci_ctx *ctx, int kernel, int precision, double *total_ms,
                      int64_t *launches, double *flops, double *bytes, const char **name);

/*
 * flops = floating-point operations one launch of kernel `kernel` executes
 * (for the MFMA opposite-spin kernel: the padded matrix tiles, i.e. the
 * alpha link count of every row rounded up to a multiple of 4 (of 16 for
 * the FP32 sigma of the slab kernel, which runs k-steps in chunks), times the
 * (pq|rs) pairs rounded up to a multiple of 16, times the beta strings
 * rounded up to the column-tile width, times 2; for the other kernels the
 * same as the algorithmic count).  Returns TBSCI_E_INVAL for a bad index,
 * precision or a NULL flops.
 */
int tbsci_timing_executed_flops(tbsci_ctx *ctx, int kernel, int precision, double *flops);

/* Message of the last failed call on this thread ("" if none). */
const char *tbsci_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TBSCI_H */
