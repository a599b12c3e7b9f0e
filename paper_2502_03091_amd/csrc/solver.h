// MG-preconditioned flexible GCR: solver buffers and the resumable outer solver.
//
// The outer FP64 flexible GCR runs a batch of right-hand-side *slots* that
// advance together one outer iteration at a time.  Every slot carries its own
// scalars, its own window of stored directions in a shared ring and its own
// stopping state, so a slot can be started (admitted) or read out (finished)
// between two iterations while the others keep running -- the basis of the
// continuously batched serving loop.  Every kernel treats each slot alone, and
// the stored directions are always summed oldest first, so a right-hand side
// gets the same iterates whichever slot it occupies and whichever others run
// beside it.
#pragma once

#include <memory>
#include <utility>
#include <vector>

#include "gcr.h"
#include "mg.h"

namespace crk {

// Device scalars of one GCR instance.
struct GcrScalars {
  DevBuf buf;
  double *sums3, *b2, *rn2, *partial, *dpart;
  double2* a;  // per-RHS minimal-residual step of the post-smoother
  int *active, *iters, *breakdown, *n_active, *level_iters;
  uint32_t* valid;
  // lazy inner solves: per iteration c_ij [kMaxCoef][nrhs][kMaxCoef], 1/||w_i||
  // and a_i [kMaxCoef][nrhs], and the solution coefficients [nrhs][kMaxCoef]
  double2 *hcoef = nullptr, *ha = nullptr, *dcoef = nullptr;
  double* hinv = nullptr;
  void alloc(int nrhs, int64_t partial_doubles, bool history = false);
};

// Pinned host int written by kernels (a polled flag), freed with its owner.
struct PinnedInt {
  int* p = nullptr;
  PinnedInt() = default;
  PinnedInt(const PinnedInt&) = delete;
  PinnedInt& operator=(const PinnedInt&) = delete;
  PinnedInt(PinnedInt&& o) noexcept : p(o.p) { o.p = nullptr; }
  PinnedInt& operator=(PinnedInt&& o) noexcept {
    std::swap(p, o.p);
    return *this;
  }
  ~PinnedInt() {
    if (p) (void)hipHostFree(p);
  }
  void alloc() {
    if (!p) CRK_HIP(hipHostMalloc(reinterpret_cast<void**>(&p), sizeof(int), hipHostMallocCoherent));
    *p = 1;
  }
};

struct LevelWork {      // coarse level l >= 1: inner solve buffers (+ post-smoother fields)
  DevBuf x, r, b, Z, W, rho, q;
  int maxit = 0;
  GcrScalars s;
  PinnedInt n_active_host;  // active RHS of the last inner iteration, for the host poll
};

struct FineWork {       // level-0 K-cycle fields in the vector precision
  DevBuf rin, rho, q;
  // post-smoother residuals of the deferred e updates: rho (q in the
  // FP16-storage form) and `defer` more fields; alpha rows of the pending
  // steps [defer][cap]
  DevBuf ring, alpha;
  int defer = 1;
};

struct OuterWork {      // FP64 outer FGCR
  DevBuf b, x, r, tmp, Z, W, mask;
  int nslots = 0;
  // Storage of the directions z_i: the K-cycle writes them into the ring in its
  // own vector precision (FP32 in the reduced forms, whose z_i are FP32 values),
  // and the FP64 operator and the solution update read them widened.
  int z_form = CRK_FORM_FP64;
  GcrScalars s;
};

// Buffers of a solve with up to `cap` right-hand sides in one form.
struct Workspace {
  int cap = -1, form = -1, restart = -1, inner = -1, coarsest = -1;
  std::vector<LevelWork> lv;  // index l (0 unused)
  FineWork fw;
  OuterWork ow;
  size_t bytes = 0;
};

std::unique_ptr<Workspace> make_workspace(Hierarchy* H, int cap, int form, const crk_solve_info& p, hipStream_t st);
bool workspace_fits(const Workspace& w, int cap, int form, const crk_solve_info& p);

enum SlotState { kSlotFree = 0, kSlotRunning = 1, kSlotConverged = 2, kSlotStopped = 3 };

class OuterSolver {
 public:
  OuterSolver(Hierarchy* H, Workspace* w, const crk_solve_info& p, hipStream_t st);

  int capacity() const { return cap_; }
  int free_slots() const;
  // Lowest free slot index, -1 if none.
  int first_free() const;
  // Start right-hand sides in slots s0 .. s0+n-1 (all free) from b_dev, a
  // complex128 host-layout device buffer [n][V][12].  Blocks on the stream.
  void admit(int s0, int n, const void* b_dev);
  // One outer iteration of every running slot.  Returns the number of slots
  // still running afterwards.
  int step();
  int running() const;
  int state(int s) const { return state_[s]; }
  int iters(int s) const { return iters_[s]; }
  // Recompute the true relative residual ||b - D x|| / ||b|| (FP64) of every
  // occupied slot.  Converged slots already carry the value of their final check.
  void refresh_residuals();
  double true_rel(int s) const { return tres_[s]; }
  // Host wall time from a slot's admission to the outer iteration at which it
  // converged or stopped (the step that decided it has synchronised the stream).
  double seconds(int s) const { return t_done_[s] - t_admit_[s]; }
  // Copy x of slots s0 .. s0+n-1 into x_dev (complex128 host layout [n][V][12]), stream ordered.
  void export_x(int s0, int n, void* x_dev);
  // Iteration counts of slots s0 .. s0+n-1: out[0] outer, out[l] summed inner iterations on level l.
  void level_iters(int s0, int n, std::vector<std::vector<int>>& out);
  void release(int s);

 private:
  Hierarchy* H_;
  Workspace* w_;
  crk_solve_info p_;
  hipStream_t st_;
  int cap_, nslots_;
  int ring_ = 0, used_ = 0;  // ring position of the next direction; stored directions
  std::vector<int> state_, iters_, nbasis_;
  std::vector<double> bn_, tres_, t_admit_, t_done_;
  DevBuf nbd_;  // per-slot window lengths for materialize
  void upload_active();
  int width() const;
  void true_residual(int width);  // tmp = b - D x over the first `width` slots, sums into s.sums3
  // Adds to x the part of the solution not applied yet: slot r's window is its
  // window[r] latest directions ending at ring slot `last` (0: nothing pending).
  void materialize(int wd, const std::vector<int>& window, int last);
};

}  // namespace crk
