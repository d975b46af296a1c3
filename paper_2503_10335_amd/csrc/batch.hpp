// Davidson solver engine: one or many TPB problems on one device, advanced
// in lock step.
//
// Every active problem ("slot") advances one Davidson iteration per round.
// A round issues each vector operation as ONE grouped launch over all slots
// that need it, the sigma builds of all slots as one grouped launch per
// kernel type (per precision), and ends with a single host synchronisation
// that brings back every slot's k x k scalars.  Slots join and leave
// between rounds, which is what the serving loop's continuous batching
// builds on; a single solve is a batch of one.
//
// One round of a slot: the Ritz pair of the current basis, its residual
// and preconditioned correction; the restart when the basis is full; two
// Gram-Schmidt passes of the correction (the subtraction of the first pass
// fused with the dot products of the second, the second with the norm);
// its sigma; the new column of the projected matrix.  The correction and
// its sigma are built before the host sees the residual of that round's
// Ritz pair, so the round in which a slot converges builds one sigma that
// is discarded.  Reductions use a block count fixed by the slot's size, so
// the arithmetic of a slot does not depend on which other slots share its
// launches.
#pragma once

#include <atomic>
#include <chrono>
#include <vector>

#include "tbsci_internal.hpp"

namespace tbsci {

constexpr int kBatchMaxVec = 16;  // largest n_max in a batch
constexpr int kBatchMaxSlots = 64;

struct BatchSlot {
    Ctx *c = nullptr;
    tbsci_davidson_opts o{};
    const double *guess = nullptr;  // optional start vector (device); no sector imposed
    // start vectors of the passes from a subspace solve (device, may be
    // null); unlike `guess` they keep the pass's sector
    const double *pass_guess[2] = {nullptr, nullptr};
    double *out = nullptr;          // optional eigenvector output (device)
    // spin-flip sector of the current pass: +1 (C^T = C), -1 (C^T = -C) or
    // 0 (none imposed); a two-sector solve runs pass 0 in +1, pass 1 in -1
    int sector = 0;
    int npass = 1, pass = 0;
    // two-sector solves without an output vector can run their sectors at
    // the same time: the primary slot (sector +1) owns a twin (sector -1)
    // with its own vectors; the engine reports the primary once both are
    // done, with the lower state
    BatchSlot *twin = nullptr;
    BatchSlot *primary = nullptr;  // set on the twin
    bool held = false;             // finished, waiting for its partner
    bool lean = false;  // 2 n_max + 3 vectors: collapse restart, no stored diagonal
    int64_t n = 0;
    int nb = 1;    // blocks of this slot in grid-stride launches
    int row = -1;  // row of the scalar area while active
    // device state: basis V / W (each from its pool of n_max + 3 vectors),
    // the latest Ritz vector kept for a hand-over or the output, the
    // diagonal, FP32 staging, partial sums
    std::vector<double *> all, vfree, wfree, V, W;
    double *X = nullptr;
    double *diag = nullptr;  // H_KK, computed in the start round
    float *f32a = nullptr, *f32b = nullptr;
    double *partial = nullptr;
    size_t bytes = 0;  // device bytes of the above (page-rounded)
    // host state
    //  kStart    start vector of a pass and its sigma
    //  kHandover mixed precision: FP64 restart from the FP32 Ritz vector
    //  kIter     one Davidson iteration
    //  kFinish   FP64 sigma of the pass's Ritz vector (energy check), and its
    //            signed copy to the output when it is the lowest so far
    enum { kStart, kHandover, kIter, kFinish, kDone } phase = kStart;
    bool fp32 = false;
    bool pass_conv = false;  // the current pass met the tolerances
    bool write_out = false;  // the finish round writes the output vector
    bool all_conv = true;    // every finished pass met the tolerances
    struct PassResult {
        bool valid = false;
        double e = 0.0, rn = 0.0, echk = 0.0;
        int sector = 0;
    } best;
    double e_other = 0.0;
    bool have_other = false;
    int k = 0;
    std::vector<double> G, y, yprev;
    double theta = 0.0, theta_prev = 0.0, rn = 1e300, best_rn = 1e300;
    int since_best = 0;
    int status = TBSCI_PENDING;
    const char *msg = "";
    tbsci_davidson_info info{};
    std::chrono::steady_clock::time_point t0;
    void *user = nullptr;  // owner's tag
    // plan of the current round
    struct Plan {
        bool sig32 = false, restart = false, took_xp = false;
        double *V0 = nullptr, *W0 = nullptr;  // start / hand-over
        double *Xn = nullptr, *WXn = nullptr, *T = nullptr, *TW = nullptr;
        bool tw_reused = false;  // lean restart: TW is a vector of the old W basis
        double *XP = nullptr, *WXP = nullptr;
        std::vector<double *> Vb, Wb;  // basis the new vector joins
    } p;
};

class BatchEngine {
  public:
    BatchEngine(int device, hipStream_t st);
    ~BatchEngine();
    BatchEngine(const BatchEngine &) = delete;
    BatchEngine &operator=(const BatchEngine &) = delete;

    // device bytes of a slot's solver state for n determinants (lean or
    // full storage; without `lean`, the mode the options ask for, full for
    // TBSCI_STORE_AUTO: an upper bound)
    static size_t slot_bytes(int64_t n, const tbsci_davidson_opts &o, bool lean);
    static size_t slot_bytes(int64_t n, const tbsci_davidson_opts &o) {
        return slot_bytes(n, o, o.storage == TBSCI_STORE_LEAN);
    }
    // allocate a slot for context c (any thread; allocation only); guess:
    // whether a start vector will be given (no sector is imposed then);
    // split: a two-sector solve gets a twin slot for its second sector
    // (solves that write no output vector only)
    static BatchSlot *make_slot(Ctx *c, const tbsci_davidson_opts &o, bool guess = false,
                                bool split = false);
    // slots a new solve adds to the engine (2 for a split solve)
    static int slots_of(const BatchSlot *s) { return s->twin ? 2 : 1; }
    // free a slot's buffers (not its context); any thread, slot not active
    static void free_slot(BatchSlot *s);

    // the slot joins at the next round (engine thread)
    void add(BatchSlot *s);
    size_t active() const { return act_.size(); }
    // one round; false if there was no active slot
    bool tick();
    // slots finished since the last call
    std::vector<BatchSlot *> take_done();
    // remove every active slot unfinished (after the stream has drained)
    std::vector<BatchSlot *> drain();

    int64_t ticks = 0;
    int max_group = 0;
    bool trace = false;

  private:
    struct Stage;
    void plan(BatchSlot &s, Stage &S);
    void commit(BatchSlot &s, const double *r, double t_sig);
    void finish(BatchSlot &s, double *keep);
    void complete(BatchSlot &s);
    void merge_twins(BatchSlot &p);

    int device_;
    hipStream_t st_;
    TableArena ar_;
    double *scal_dev_ = nullptr, *scal_host_ = nullptr;
    hipEvent_t ev_[2] = {nullptr, nullptr};
    std::vector<BatchSlot *> act_, done_;
    std::vector<int> free_rows_;
};

// Solve one problem (guess and out optional, device FP64 [l_alpha][l_beta]);
// abort, when set, ends the solve at the next round with TBSCI_E_STATE.
int solve_one(Ctx &c, const tbsci_davidson_opts &o, const double *guess, double *out,
              tbsci_davidson_info &info, hipStream_t st,
              const std::atomic<bool> *abort = nullptr);

}  // namespace tbsci
