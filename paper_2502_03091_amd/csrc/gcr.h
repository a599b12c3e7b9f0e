// Multi-RHS flexible GCR kernels: interface.
#pragma once

#include "blas.h"
#include "common.h"

namespace crk {

constexpr int kMaxBasis = 32;  // directions per multidot pass (and per outer GCR cycle)
constexpr int kMaxCoef = 64;   // stored directions of an inner GCR (coefficient stride)

// nrhs vectors of n complex entries; entry e of rhs r at r*rs + e*es.
struct FieldShape {
  int64_t n;
  int nrhs;
  int64_t rs, es;
  int64_t total() const { return n * nrhs; }
};

inline FieldShape fine_shape(int64_t V, int nrhs) { return FieldShape{12 * V, nrhs, 12 * V, 1}; }
inline FieldShape coarse_shape(int64_t V, int N, int nrhs) { return FieldShape{int64_t(N) * V, nrhs, 1, nrhs}; }

// Rows of the partial buffers (times nrhs * 2*kMaxBasis doubles for multidot);
// inner: rhs-inner (coarse) layout.
int64_t gcr_partial_rows(int64_t n, bool inner);

void gcr_multidot(int prec, const void* W, int64_t fstride, int nj, const void* w, const FieldShape& f, double* partial,
                  const uint32_t* valid, double2* coef, hipStream_t st);
// The solvers keep the preconditioned directions z_i as they are and form the
// solution from them when it is needed (lazy): an iteration only
// orthogonalises w_i against the stored directions (classical Gram-Schmidt,
// summed cyclically from slot j_first, the oldest), normalises it, updates r
// (with the <w_i, r>, ||w_i||^2 partials dpart of dnch chunks from
// rhs_dot_launch, reduced inside every workgroup), and records c_ij (the
// multidot's coef), 1/||w_i|| (hinv[r]) and a_i (ha[r]); rn2 (optional)
// receives ||r||^2.
void gcr_multiaxpy_w(int prec, const void* W, int64_t fstride, int nj, int j_first, void* w, const double2* coef,
                     const FieldShape& f, hipStream_t st);
void gcr_update_lazy(int prec, void* w, void* r, const double* dpart, int64_t dnch, const int* active, int* breakdown,
                     const FieldShape& f, double* partial, double* rn2, double* hinv, double2* ha, hipStream_t st);
// The same step in one pass for rhs-inner (coarse) fields, one RHS included
// (gcr_one_pass_shape): dpart holds the <w_i, r>, ||w_i||^2 partials of the
// unmodified w_i, coef the multidot's c_ij (not read for nj = 0); ||w^||^2 and
// <w^, r> follow from them (orthonormal stored directions, r orthogonal to
// them), so w_i is orthogonalised, normalised and r updated in one kernel.
// partial receives the ||r||^2 partials of the check, in the rhs-inner
// chunks whatever the RHS count; returns their number of rows (gcr_check's
// partial_rows).
bool gcr_one_pass_shape(const FieldShape& f);
// One-pass step on rhs-outer fields over a ring of nj (>= 0) stored directions
// (summed from slot j_first on, oldest first; zero coefficients skipped):
// w^ = w - sum c_j W_j with ||w^||^2 = ||w||^2 - sum |c_j|^2 and
// <w^, r> = <w, r> from dpart (the dots of the unmodified w), w <- w^/||w^||,
// r -= a w, ||r||^2 reduced into rn2 (if not NULL); hinv, ha as gcr_update_lazy.
void gcr_gs_update_ring(int prec, const void* W, int64_t fstride, int nj, int j_first, void* w, void* r,
                        const double2* coef, const double* dpart, int64_t dnch, const int* active, int* breakdown,
                        const FieldShape& f, double* partial, double* rn2, double* hinv, double2* ha, hipStream_t st);
int64_t gcr_gs_update(int prec, const void* W, int64_t fstride, int nj, void* w, void* r, const double2* coef,
                   const double* dpart, int64_t dnch, const int* active, int* breakdown, const FieldShape& f,
                   double* partial, double* hinv, double2* ha, hipStream_t st);
// Inner solve of K iterations with records c_ij at hcoef[i][nrhs][kMaxCoef],
// 1/||w_i|| and a_i at hinv/ha[i][nrhs]:
// x = sum_{i<K} d_i z_i with the d_i of the recorded recursion (dcoef: [nrhs][kMaxCoef] work space).
void gcr_lazy_solution(int prec, const void* Z, int64_t fstride, int K, void* x, const double2* hcoef,
                       const double* hinv, const double2* ha, double2* dcoef, const FieldShape& f, hipStream_t st);
// Outer (FP64, rhs-outer) lazy form over a ring of nslots directions: RHS r's
// window is its nb[r] (device) latest directions ending at ring slot last;
// records are [slot][cap] (c: [slot][cap][kMaxCoef]).  Adds the not yet
// applied part of the solution, sum over the window of a_i p_i, to x and
// clears those a_i.  z_form: storage of the directions (FP64, or FP32 when
// they hold FP32 values: the K-cycle output of the reduced-precision forms).
void gcr_ring_materialize(const void* Z, int z_form, int64_t fstride, const int* nb, int last, int nslots, int cap,
                          void* x, const double2* hcoef, const double* hinv, double2* ha, double2* dcoef,
                          const FieldShape& f, hipStream_t st);
// n_active_host (optional): pinned host memory that also receives the count of active RHS;
// partial_rows (optional): rows of partial, when not the field shape's own chunking.
void gcr_check(const double* partial, const FieldShape& f, double tol2, const double* b2, const int* breakdown,
               int* active, int* iters, double* rn2, int* n_active, int* level_iters, hipStream_t st,
               int* n_active_host = nullptr, int64_t partial_rows = -1);
void gcr_start(const double* sums3, int nrhs, double* b2, int* active, int* iters, int* n_active, hipStream_t st);
void field_axpby(int prec, const void* x, void* y, double a, double b, int64_t total, hipStream_t st);
// out = a x + b y, out separate from y (or equal to it)
void field_axpby_to(int prec, const void* x, const void* y, void* out, double a, double b, int64_t total,
                    hipStream_t st);
void field_masked_copy(int prec, const void* x, void* y, const int* mask, const FieldShape& f, hipStream_t st);

}  // namespace crk
