// Per-RHS BLAS-1 launchers (see blas.hip).
#pragma once

#include <utility>
#include <vector>

#include "common.h"

namespace crk {

// Reductions over rhs-inner fields (element e of rhs r at e*nrhs + r) use
// workgroup chunks of kInnerChunk elements of one RHS (one per thread): one
// partial per (chunk, rhs), so an RHS's sums do not depend on how many RHS
// share the field.
constexpr int kInnerChunk = 256;

// Number of partial rows rhs_dot needs per RHS for vectors of n entries
// (partial buffer: rhs_dot_partials(n, inner) * nrhs * 3 doubles).
int64_t rhs_dot_partials(int64_t n, bool inner);

// out3[r] = (Re, Im) of sum_e conj(a) b, and sum_e |a|^2, for every rhs r;
// entry e of rhs r at index r*rs + e*es.  b may be NULL (then b = a).
// prec: CRK_FORM_FP64 (double2 data) or CRK_FORM_FP32 (float2 data).
void rhs_dot(int prec, const void* a, const void* b, int64_t n, int nrhs, int64_t rs, int64_t es, double* partial,
             double* out3, hipStream_t st);

// Launch only the partial-sum pass of rhs_dot: partial[chunk][r][3]; returns the number of chunks.
int64_t rhs_dot_launch(int prec, const void* a, const void* b, int64_t n, int nrhs, int64_t rs, int64_t es,
                       double* partial, hipStream_t st);

void reduce_partials(const double* partial, int64_t nchunk, int nrhs, int nv, double* out, hipStream_t st);

// alpha[r] = <q,r>/<q,q> from sums3[r] = (Re<q,r>, Im<q,r>, <q,q>), 0 when <q,q> = 0.
void mr_alpha(const double* sums3, int nrhs, double2* alpha, hipStream_t st);

// psi += alpha r; r -= alpha q (n entries per rhs; rhs-outer or rhs-inner layout).
// update_r = false: psi only, for the last step of a smoother whose residual is
// not used afterwards (q is then not read and r not written).
void mr_update(int prec, void* psi, void* r, const void* q, const double2* alpha, int64_t n, int nrhs, bool rhs_inner,
               hipStream_t st, bool update_r = true);
// The same update on the fine level with psi in FP32 and r, q in FP16 storage
// (AoSoA fine fields of V sites, one scale per site and RHS; r is rescaled).
void mr_update_fine_h(void* psi, void* r, const void* q, const double2* alpha, int64_t V, int nrhs, hipStream_t st,
                      bool update_r = true);

// MR updates of several sweeps applied to psi in one pass.  Each sweep k still
// forms its residual r_{k+1} = r_k - alpha_k q_k, into a field of its own, but
// psi is read and written only when the pending sweeps are flushed:
// psi += alpha_j r_j for the pending sweeps j in order.  Per element this is
// the sequence of fused multiply-adds of one mr_update per sweep, so the
// result is bitwise the same; each sweep moves r, q in and r out, and a flush
// adds psi in and out and the older pending residuals in.
constexpr int kMrMaxDefer = 8;
struct MrPending {
  const void* r[kMrMaxDefer];        // r_j of the pending sweeps, oldest first; the last is the current r_k
  const double2* alpha[kMrMaxDefer];  // their alpha_j [nrhs]
  int n;                              // pending sweeps (>= 1)
};
// rnext = r_k - alpha_k q (skipped when rnext is null); when psi is not null,
// psi += alpha_j r_j over all pending sweeps.  Layouts as mr_update.
void mr_update_ring(int prec, void* psi, const MrPending& pend, const void* q, void* rnext, int64_t n, int nrhs,
                    bool rhs_inner, hipStream_t st);

// Host side of one run of MR sweeps with psi updates deferred over D sweeps:
// the residual of sweep k lives in slot k mod (D + 1) and its alpha in row
// k mod D of `alpha` (rows `alpha_stride` apart).  One slot means D = 1, the
// in-place update of mr_update.  Use one object per run of sweeps.
class MrSweeps {
 public:
  MrSweeps(std::vector<void*> slots, double2* alpha, size_t alpha_stride)
      : slots_(std::move(slots)), alpha_(alpha), stride_(alpha_stride),
        D_(slots_.size() > 1 ? int(slots_.size()) - 1 : 1) {}
  void* r(int it) const { return slots_[size_t(it) % slots_.size()]; }
  double2* alpha(int it) const { return alpha_ + size_t(it % D_) * stride_; }
  // After sweep `it` of `nsweeps` formed q = D r(it) and alpha(it): the psi
  // updates that are due and r(it + 1) (not formed after the last sweep).
  void update(int prec, void* psi, const void* q, int it, int nsweeps, int64_t n, int nrhs, bool rhs_inner,
              hipStream_t st);
  // The same for the fine level with psi in FP32 and r, q in FP16 storage
  // (the arithmetic of mr_update_fine_h).
  void update_fine_h(void* psi, const void* q, int it, int nsweeps, int64_t V, int nrhs, hipStream_t st);

 private:
  std::vector<void*> slots_;
  double2* alpha_;
  size_t stride_;
  int D_;
  int pending_ = 0;
};

// v[e*nrhs + r] *= f[r] for n entries per rhs (rhs-inner layout).
void scale_rhs_inner(int prec, void* v, const double* f, int64_t n, int nrhs, hipStream_t st);

// out[i] = 1/sqrt(sums[i*nv + comp]) (0 for a zero sum).
void inv_sqrt(const double* sums, int nv, int comp, int n, double* out, hipStream_t st);

// total complex Gaussian entries from Philox4x32-10 (counter = entry index, stream).
void gaussian_fill(int prec, void* out, int64_t total, uint64_t seed, uint32_t stream, hipStream_t st);

}  // namespace crk
