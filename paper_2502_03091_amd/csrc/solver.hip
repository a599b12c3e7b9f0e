// MG-preconditioned flexible GCR (paper, Sec. 2 last paragraph: the hierarchy
// is used as a K-cycle preconditioner of a flexible outer solver).
//
// Outer: flexible GCR in FP64 on the fine level, restart m_r, stopping on the
// TRUE residual ||b - D x|| / ||b|| (recomputed when the recursive residual
// claims convergence and at every restart -- iterative refinement for the
// reduced-precision forms).  Preconditioner: one K-cycle in the solve form
// (FP64, or FP32 vectors with FP32 or FP16-storage operators):
//   r_c = P^dag r;  e_c = FGCR on D_{l+1} to relative tau or N iterations,
//   itself preconditioned by the next level's cycle (the coarsest level runs
//   plain GCR);  e = P e_c;  nu_post MR steps on D_l e = r.
// All right-hand sides advance together; per-RHS scalars, active flags and a
// ring of stored directions with per-RHS valid windows reproduce, RHS by RHS,
// the single-RHS recursion.
#include <chrono>

#include "solver.h"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "blas.h"
#include "coarse.h"

namespace crk {

void GcrScalars::alloc(int nrhs, int64_t partial_doubles, bool history) {
  const size_t nr = size_t(nrhs);
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off += (b + 255) & ~size_t(255); return o; };
  const size_t o_s3 = take(sizeof(double) * 3 * nr), o_b2 = take(sizeof(double) * nr),
               o_rn = take(sizeof(double) * nr), o_a = take(sizeof(double2) * nr),
               o_act = take(sizeof(int) * nr), o_it = take(sizeof(int) * nr), o_bd = take(sizeof(int) * nr),
               o_na = take(sizeof(int)), o_li = take(sizeof(int) * nr), o_val = take(sizeof(uint32_t) * nr),
               o_part = take(sizeof(double) * size_t(partial_doubles)),
               o_dpart = take(sizeof(double) * size_t(partial_doubles));
  const size_t nh = history ? size_t(kMaxCoef) : 0;
  const size_t o_hc = take(sizeof(double2) * nh * nr * kMaxCoef), o_hi = take(sizeof(double) * nh * nr),
               o_ha = take(sizeof(double2) * nh * nr), o_dc = take(sizeof(double2) * (history ? nr : 0) * kMaxCoef);
  buf.alloc(off);
  char* c = static_cast<char*>(buf.p);
  sums3 = reinterpret_cast<double*>(c + o_s3);
  b2 = reinterpret_cast<double*>(c + o_b2);
  rn2 = reinterpret_cast<double*>(c + o_rn);
  a = reinterpret_cast<double2*>(c + o_a);
  active = reinterpret_cast<int*>(c + o_act);
  iters = reinterpret_cast<int*>(c + o_it);
  breakdown = reinterpret_cast<int*>(c + o_bd);
  n_active = reinterpret_cast<int*>(c + o_na);
  level_iters = reinterpret_cast<int*>(c + o_li);
  valid = reinterpret_cast<uint32_t*>(c + o_val);
  partial = reinterpret_cast<double*>(c + o_part);
  dpart = reinterpret_cast<double*>(c + o_dpart);
  hcoef = history ? reinterpret_cast<double2*>(c + o_hc) : nullptr;
  hinv = history ? reinterpret_cast<double*>(c + o_hi) : nullptr;
  ha = history ? reinterpret_cast<double2*>(c + o_ha) : nullptr;
  dcoef = history ? reinterpret_cast<double2*>(c + o_dc) : nullptr;
}

namespace {

constexpr int kPollEvery = 4;

int64_t partial_doubles(int64_t n, int nrhs, bool inner) {
  const int64_t a = gcr_partial_rows(n, inner) * nrhs * 2 * kMaxBasis;
  const int64_t b = rhs_dot_partials(n, inner) * nrhs * 3;
  const int64_t c = wilson_partial_blocks(n / 12 + 1) * nrhs * 3;
  return std::max(a, std::max(b, c));
}

int vec_prec(int form) { return form == CRK_FORM_FP64 ? CRK_FORM_FP64 : CRK_FORM_FP32; }
size_t vec_bytes(int form) { return form == CRK_FORM_FP64 ? sizeof(double2) : sizeof(float2); }
// Operator storage used on the fine level in a form (vectors there are FP32 for FP16S).
int fine_op_form(int form) { return form == CRK_FORM_FP64 ? CRK_FORM_FP64 : CRK_FORM_FP32; }
int ring_slots(const crk_solve_info& p) { return std::max(1, std::min(p.restart, p.max_iter)); }
// Steps of the fine post-smoother whose e updates share one pass.
int post_defer(int nlev, const crk_solve_info& p) {
  if (nlev <= 1) return 1;
  return std::max(1, std::min(p.post_defer > 0 ? p.post_defer : 4, p.nu_post));
}
// Storage of the outer directions z_i: the K-cycle's own vector storage (FP32
// for the reduced forms), FP64 in the plain form and without coarse levels.
int outer_z_form(const Hierarchy* H, int form) {
  return H->nlev > 1 && form != CRK_FORM_FP64 ? CRK_FORM_FP32 : CRK_FORM_FP64;
}

FieldShape shape(Hierarchy* H, int l, int nrhs) {
  return l == 0 ? fine_shape(H->V(0), nrhs) : coarse_shape(H->V(l), H->N(l), nrhs);
}

void kcycle(Hierarchy* H, Workspace& w, int l, const crk_solve_info& p, int nrhs, const void* rin, void* eout,
            hipStream_t st);

// Inner flexible GCR on coarse level l over the first nrhs RHS: solves D_l x = b (lw.b) from x = 0.
void inner_fgcr(Hierarchy* H, Workspace& w, int l, const crk_solve_info& p, int nrhs, hipStream_t st) {
  LevelWork& lw = w.lv[l];
  const int form = w.form, prec = vec_prec(form);
  const FieldShape f = shape(H, l, nrhs);
  const int64_t fs = f.total();  // complex entries per stored field
  const size_t fb = vec_bytes(form) * size_t(fs);
  GcrScalars& s = lw.s;
  CRK_HIP(hipMemcpyAsync(lw.r.p, lw.b.p, fb, hipMemcpyDeviceToDevice, st));
  rhs_dot(prec, lw.b.p, nullptr, f.n, nrhs, f.rs, f.es, s.partial, s.sums3, st);
  gcr_start(s.sums3, nrhs, s.b2, s.active, s.iters, s.n_active, st);
  const double tol2 = p.tau * p.tau;
  const bool precond = l < H->nlev - 1;
  char* Z = static_cast<char*>(lw.Z.p);
  char* W = static_cast<char*>(lw.W.p);
  int n_active = 1, K = 0;
  for (int i = 0; i < lw.maxit; ++i) {
    void* zi = Z + fb * i;
    void* wi = W + fb * i;
    if (precond) {
      kcycle(H, w, l, p, nrhs, lw.r.p, zi, st);
      level_apply(H, l, form, zi, wi, nrhs, st);
    } else {
      // unpreconditioned: z_i = r, stored by the operator launch that computes w_i = D r
      level_apply(H, l, form, lw.r.p, wi, nrhs, st, nullptr, false, zi);
    }
    // z_i stays as the preconditioner (or the copy of r) left it: only w_i is
    // orthogonalised and normalised, and the solution is formed after the loop
    double2* ci = s.hcoef + size_t(i) * nrhs * kMaxCoef;
    int64_t rows = -1;  // partial rows of the check: the field's own chunking unless set
    if (gcr_one_pass_shape(f)) {
      // coefficients and the dots of the unmodified w_i, then one pass
      if (i > 0) gcr_multidot(prec, W, fs, i, wi, f, s.partial, nullptr, ci, st);
      const int64_t dn = rhs_dot_launch(prec, wi, lw.r.p, f.n, nrhs, f.rs, f.es, s.dpart, st);
      rows = gcr_gs_update(prec, W, fs, i, wi, lw.r.p, ci, s.dpart, dn, s.active, s.breakdown, f, s.partial,
                           s.hinv + size_t(i) * nrhs, s.ha + size_t(i) * nrhs, st);
    } else {
      if (i > 0) {
        gcr_multidot(prec, W, fs, i, wi, f, s.partial, nullptr, ci, st);
        gcr_multiaxpy_w(prec, W, fs, i, 0, wi, ci, f, st);
      }
      const int64_t dn = rhs_dot_launch(prec, wi, lw.r.p, f.n, nrhs, f.rs, f.es, s.dpart, st);
      gcr_update_lazy(prec, wi, lw.r.p, s.dpart, dn, s.active, s.breakdown, f, s.partial, nullptr,
                      s.hinv + size_t(i) * nrhs, s.ha + size_t(i) * nrhs, st);
    }
    gcr_check(s.partial, f, tol2, s.b2, s.breakdown, s.active, s.iters, s.rn2, s.n_active, s.level_iters, st,
              lw.n_active_host.p, rows);
    K = i + 1;
    // Converged RHS are frozen on the device; the host only polls every few
    // iterations to stop launching once every RHS is done (the check kernel
    // writes the count to pinned host memory, so a poll is a stream wait only).
    if ((i + 1) % kPollEvery == 0 || i + 1 == lw.maxit) {
      CRK_HIP(hipStreamSynchronize(st));
      n_active = *static_cast<volatile int*>(lw.n_active_host.p);
      if (n_active == 0) break;
    }
  }
  gcr_lazy_solution(prec, Z, fs, K, lw.x.p, s.hcoef, s.hinv, s.ha, s.dcoef, f, st);
}

void kcycle(Hierarchy* H, Workspace& w, int l, const crk_solve_info& p, int nrhs, const void* rin, void* eout,
            hipStream_t st) {
  const int form = w.form, prec = vec_prec(form);
  const int opf = l == 0 ? fine_op_form(form) : form;
  LevelWork& nx = w.lv[l + 1];
  level_restrict(H, l, form, rin, nx.b.p, nrhs, st);
  inner_fgcr(H, w, l + 1, p, nrhs, st);
  level_prolong(H, l, form, nx.x.p, eout, nrhs, false, st);
  if (p.nu_post <= 0) return;
  // MR on D_l e = r, starting from e:  rho = r - D e ; q = D rho ; e += alpha rho ; rho -= alpha q
  if (l == 0 && form == CRK_FORM_FP16S) {
    // FP16-storage form on the fine level: e (the cycle's output) stays FP32,
    // the MR residual rho and q = D rho are held in FP16 storage (one scale per
    // site and RHS) and the fine operator reads and writes them in that form.
    const int64_t V0 = H->V(0);
    void* r32 = w.fw.rho.p;
    level_residual(H, 0, CRK_FORM_FP32, eout, rin, r32, nrhs, st);  // r32 = rin - D e
    void* rhoh = w.fw.q.p;
    void* qh = w.fw.rho.p;  // r32 is no longer needed once converted (stream order)
    field_convert(CRK_FORM_FP32, r32, CRK_FORM_FP16S, rhoh, V0, 12, nrhs, st);
    GcrScalars& s0 = w.ow.s;
    // the e updates of up to four sweeps share one pass (residuals in a ring)
    std::vector<void*> slots{rhoh};
    const size_t fv = vec_bytes(form) * 12 * size_t(V0) * w.cap;  // each ring field holds an FP16 field set
    for (int j = 0; w.fw.defer > 1 && j < w.fw.defer; ++j) slots.push_back(static_cast<char*>(w.fw.ring.p) + fv * j);
    MrSweeps mr(slots, slots.size() > 1 ? w.fw.alpha.as<double2>() : s0.a, size_t(w.cap));
    for (int it = 0; it < p.nu_post; ++it) {
      level_apply(H, 0, CRK_FORM_FP16S, mr.r(it), qh, nrhs, st, s0.partial);
      reduce_partials(s0.partial, wilson_partial_blocks(V0), nrhs, 3, s0.sums3, st);
      mr_alpha(s0.sums3, nrhs, mr.alpha(it), st);
      mr.update_fine_h(eout, qh, it, p.nu_post, V0, nrhs, st);  // last step: e only
    }
    return;
  }
  const FieldShape f = shape(H, l, nrhs);
  void* q = l == 0 ? w.fw.q.p : w.lv[l].q.p;
  GcrScalars& s = l == 0 ? w.ow.s : w.lv[l].s;
  // the scalars of level l are idle while its K-cycle runs (the cycle is called
  // between the solver's kernel phases); only sums3/partial/a are reused here.
  // On the fine level the e updates of up to four sweeps share one pass.
  std::vector<void*> slots{l == 0 ? w.fw.rho.p : w.lv[l].rho.p};
  if (l == 0 && w.fw.defer > 1) {
    const size_t fv = vec_bytes(form) * 12 * size_t(H->V(0)) * w.cap;
    for (int j = 0; j < w.fw.defer; ++j) slots.push_back(static_cast<char*>(w.fw.ring.p) + fv * j);
  }
  MrSweeps mr(slots, slots.size() > 1 ? w.fw.alpha.as<double2>() : s.a, size_t(w.cap));
  level_residual(H, l, opf, eout, rin, mr.r(0), nrhs, st);  // rho = rin - D e
  for (int it = 0; it < p.nu_post; ++it) {
    if (l == 0) {
      level_apply(H, 0, opf, mr.r(it), q, nrhs, st, s.partial);
      reduce_partials(s.partial, wilson_partial_blocks(H->V(0)), nrhs, 3, s.sums3, st);
    } else {
      level_apply(H, l, opf, mr.r(it), q, nrhs, st);
      rhs_dot(prec, q, mr.r(it), f.n, nrhs, f.rs, f.es, s.partial, s.sums3, st);
    }
    mr_alpha(s.sums3, nrhs, mr.alpha(it), st);
    mr.update(prec, eout, q, it, p.nu_post, f.n, nrhs, l > 0, st);  // last step: e only
  }
}

void validate(Hierarchy* H, const crk_solve_info& p) {
  CRK_REQUIRE(p.tol > 0 && std::isfinite(p.tol), "tol must be > 0");
  CRK_REQUIRE(p.max_iter >= 1, "max_iter must be >= 1");
  CRK_REQUIRE(p.restart >= 1 && p.restart <= kMaxBasis, "restart must be in [1, 32]");
  CRK_REQUIRE(p.inner_maxit >= 1 && p.inner_maxit <= kMaxBasis, "inner_maxit must be in [1, 32]");
  CRK_REQUIRE(p.coarsest_maxit >= 1 && p.coarsest_maxit <= 64, "coarsest_maxit must be in [1, 64]");
  CRK_REQUIRE(p.form == CRK_FORM_FP64 || p.form == CRK_FORM_FP32 || p.form == CRK_FORM_FP16S, "unknown form");
  CRK_REQUIRE(p.tau > 0 && p.nu_post >= 0, "tau must be > 0 and nu_post >= 0");
  CRK_REQUIRE(p.post_defer >= 0 && p.post_defer <= kMrMaxDefer, "post_defer must be in [0, 8]");
  (void)H;
}

}  // namespace

bool workspace_fits(const Workspace& w, int cap, int form, const crk_solve_info& p) {
  return w.cap >= cap && w.form == form && w.restart == ring_slots(p) && w.inner == p.inner_maxit &&
         w.coarsest == p.coarsest_maxit && w.fw.defer == post_defer(int(w.lv.size()), p);
}

std::unique_ptr<Workspace> make_workspace(Hierarchy* H, int cap, int form, const crk_solve_info& p, hipStream_t st) {
  validate(H, p);
  CRK_REQUIRE(cap >= 1 && cap <= 64, "right-hand-side capacity must be in [1, 64]");
  auto wp = std::make_unique<Workspace>();
  Workspace& w = *wp;
  const int nslots = ring_slots(p);
  w.cap = cap;
  w.form = form;
  w.restart = nslots;
  w.inner = p.inner_maxit;
  w.coarsest = p.coarsest_maxit;
  const int64_t V0 = H->V(0);
  const size_t f64 = sizeof(double2) * 12 * size_t(V0) * cap;
  OuterWork& o = w.ow;
  o.nslots = nslots;
  o.z_form = outer_z_form(H, form);
  const size_t zslot = vec_bytes(o.z_form) * 12 * size_t(V0) * cap;
  o.b.alloc(f64); o.x.alloc(f64); o.r.alloc(f64); o.tmp.alloc(f64);
  o.Z.alloc(zslot * nslots); o.W.alloc(f64 * nslots);
  o.mask.alloc(sizeof(int) * cap);
  o.s.alloc(cap, partial_doubles(12 * V0, cap, false), true);
  // Slots may start at any ring position: every stored direction a slot's
  // kernels touch must hold finite values from the start.
  CRK_HIP(hipMemsetAsync(o.Z.p, 0, zslot * nslots, st));
  CRK_HIP(hipMemsetAsync(o.W.p, 0, f64 * nslots, st));
  CRK_HIP(hipMemsetAsync(o.x.p, 0, f64, st));
  CRK_HIP(hipMemsetAsync(o.r.p, 0, f64, st));
  CRK_HIP(hipMemsetAsync(o.b.p, 0, f64, st));
  w.bytes += f64 * (4 + size_t(nslots)) + zslot * nslots;
  if (H->nlev > 1) {
    const size_t fv = vec_bytes(form) * 12 * size_t(V0) * cap;
    w.fw.rin.alloc(fv); w.fw.rho.alloc(fv); w.fw.q.alloc(fv);
    w.bytes += 3 * fv;
    w.fw.defer = post_defer(H->nlev, p);
    if (w.fw.defer > 1) {
      w.fw.ring.alloc(fv * w.fw.defer);
      w.fw.alpha.alloc(sizeof(double2) * w.fw.defer * cap);
      w.bytes += fv * w.fw.defer;
    }
  }
  w.lv.resize(H->nlev);
  for (int l = 1; l < H->nlev; ++l) {
    LevelWork& lw = w.lv[l];
    lw.maxit = l == H->nlev - 1 ? p.coarsest_maxit : p.inner_maxit;
    CRK_REQUIRE(lw.maxit <= 64, "coarsest basis too large");
    const size_t cv = vec_bytes(form) * size_t(H->N(l)) * H->V(l) * cap;
    lw.x.alloc(cv); lw.r.alloc(cv); lw.b.alloc(cv);
    if (l < H->nlev - 1) { lw.rho.alloc(cv); lw.q.alloc(cv); w.bytes += 2 * cv; }
    lw.Z.alloc(cv * lw.maxit); lw.W.alloc(cv * lw.maxit);
    lw.s.alloc(cap, partial_doubles(int64_t(H->N(l)) * H->V(l), cap, true), true);
    lw.n_active_host.alloc();
    CRK_HIP(hipMemsetAsync(lw.s.level_iters, 0, sizeof(int) * cap, st));
    w.bytes += cv * (3 + 2 * size_t(lw.maxit));
  }
  CRK_HIP(hipStreamSynchronize(st));
  return wp;
}

// ------------------------------------------------------------------ outer solver

OuterSolver::OuterSolver(Hierarchy* H, Workspace* w, const crk_solve_info& p, hipStream_t st)
    : H_(H), w_(w), p_(p), st_(st), cap_(w->cap), nslots_(w->ow.nslots) {
  validate(H, p);
  CRK_REQUIRE(workspace_fits(*w, 1, p.form, p), "workspace does not match the solve parameters");
  state_.assign(cap_, kSlotFree);
  iters_.assign(cap_, 0);
  nbasis_.assign(cap_, 0);
  bn_.assign(cap_, 0.0);
  tres_.assign(cap_, 0.0);
  t_admit_.assign(cap_, 0.0);
  t_done_.assign(cap_, 0.0);
  nbd_.alloc(sizeof(int) * size_t(cap_));
}

namespace {
double wall_now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

int OuterSolver::free_slots() const { return int(std::count(state_.begin(), state_.end(), int(kSlotFree))); }

int OuterSolver::first_free() const {
  for (int s = 0; s < cap_; ++s)
    if (state_[s] == kSlotFree) return s;
  return -1;
}

int OuterSolver::running() const { return int(std::count(state_.begin(), state_.end(), int(kSlotRunning))); }

int OuterSolver::width() const {
  for (int s = cap_ - 1; s >= 0; --s)
    if (state_[s] != kSlotFree) return s + 1;
  return 0;
}

void OuterSolver::upload_active() {
  std::vector<int> a(cap_);
  for (int s = 0; s < cap_; ++s) a[s] = state_[s] == kSlotRunning;
  CRK_HIP(hipMemcpyAsync(w_->ow.s.active, a.data(), sizeof(int) * cap_, hipMemcpyHostToDevice, st_));
  CRK_HIP(hipStreamSynchronize(st_));  // the host vector goes out of scope
}

void OuterSolver::admit(int s0, int n, const void* b_dev) {
  CRK_REQUIRE(n >= 1 && s0 >= 0 && s0 + n <= cap_, "slot range out of bounds");
  for (int s = s0; s < s0 + n; ++s) CRK_REQUIRE(state_[s] == kSlotFree, "slot is in use");
  OuterWork& o = w_->ow;
  GcrScalars& s = o.s;
  const int64_t V = H_->V(0);
  const int64_t per = 12 * V;  // complex entries per RHS
  double2* b = o.b.as<double2>() + per * s0;
  double2* x = o.x.as<double2>() + per * s0;
  double2* r = o.r.as<double2>() + per * s0;
  const size_t bytes = sizeof(double2) * size_t(per) * n;
  field_import(CRK_FORM_FP64, static_cast<const double2*>(b_dev), b, H_->fine_geo.pos.as<int>(), V, 12, n, st_);
  CRK_HIP(hipMemsetAsync(x, 0, bytes, st_));
  CRK_HIP(hipMemcpyAsync(r, b, bytes, hipMemcpyDeviceToDevice, st_));
  for (int j = 0; j < nslots_; ++j)  // no solution part of an earlier occupant is pending in these slots
    CRK_HIP(hipMemsetAsync(s.ha + size_t(j) * cap_ + s0, 0, sizeof(double2) * size_t(n), st_));
  for (int l = 1; l < H_->nlev; ++l)
    CRK_HIP(hipMemsetAsync(w_->lv[l].s.level_iters + s0, 0, sizeof(int) * n, st_));
  rhs_dot(CRK_FORM_FP64, b, nullptr, per, n, per, 1, s.partial, s.sums3, st_);
  std::vector<double> h3(3 * size_t(n));
  CRK_HIP(hipMemcpyAsync(h3.data(), s.sums3, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, st_));
  CRK_HIP(hipStreamSynchronize(st_));
  for (int i = 0; i < n; ++i) {
    const int q = s0 + i;
    bn_[q] = std::sqrt(h3[3 * i + 2]);
    CRK_REQUIRE(std::isfinite(bn_[q]), "right-hand side is not finite");
    iters_[q] = 0;
    nbasis_[q] = 0;
    tres_[q] = 0.0;
    state_[q] = bn_[q] > 0 ? kSlotRunning : kSlotConverged;  // b = 0: x = 0 is exact
    t_admit_[q] = wall_now();
    t_done_[q] = t_admit_[q];
  }
  upload_active();
}

void OuterSolver::true_residual(int wd) {
  OuterWork& o = w_->ow;
  GcrScalars& s = o.s;
  const FieldShape f = fine_shape(H_->V(0), wd);
  level_apply(H_, 0, CRK_FORM_FP64, o.x.p, o.tmp.p, wd, st_);
  field_axpby(CRK_FORM_FP64, o.b.p, o.tmp.p, 1.0, -1.0, f.total(), st_);
  rhs_dot(CRK_FORM_FP64, o.tmp.p, nullptr, f.n, wd, f.rs, f.es, s.partial, s.sums3, st_);
}

int OuterSolver::step() {
  const int wd = width();
  if (running() == 0) return 0;
  std::vector<char> was_running(wd);
  for (int r = 0; r < wd; ++r) was_running[r] = state_[r] == kSlotRunning;
  Workspace& w = *w_;
  OuterWork& o = w.ow;
  GcrScalars& s = o.s;
  const int64_t V = H_->V(0);
  const FieldShape f = fine_shape(V, wd);
  const int64_t fcap = 12 * V * cap_;  // complex entries between stored directions
  const size_t fbcap = sizeof(double2) * size_t(fcap);
  char* Z = static_cast<char*>(o.Z.p);
  char* W = static_cast<char*>(o.W.p);
  void* zi = Z + vec_bytes(o.z_form) * size_t(fcap) * ring_;
  void* wi = W + fbcap * ring_;
  if (H_->nlev > 1) {
    void* rin = o.r.p;
    if (p_.form != CRK_FORM_FP64) {
      field_convert(CRK_FORM_FP64, o.r.p, CRK_FORM_FP32, w.fw.rin.p, V, 12, wd, st_);
      rin = w.fw.rin.p;
    }
    kcycle(H_, w, 0, p_, wd, rin, zi, st_);  // z_i in the ring, in the cycle's vector storage
  } else {
    CRK_HIP(hipMemcpyAsync(zi, o.r.p, sizeof(double2) * size_t(f.total()), hipMemcpyDeviceToDevice, st_));
  }
  level_apply(H_, 0, CRK_FORM_FP64, zi, wi, wd, st_, nullptr, false, nullptr, o.z_form);
  used_ = std::min(used_ + 1, nslots_);
  // Lazy form: z_i stays as the K-cycle returned it, only w_i is orthogonalised
  // and normalised; c_ij, 1/||w_i|| and a_i are recorded per ring slot and the
  // solution is brought up to date (materialize) whenever it is needed.
  double2* ci = s.hcoef + size_t(ring_) * cap_ * kMaxCoef;
  std::vector<uint32_t> valid(wd, 0);  // read by a copy on the stream: lives until the sync below
  if (used_ > 1) {
    for (int r = 0; r < wd; ++r)
      for (int a = 1; a <= nbasis_[r]; ++a) valid[r] |= 1u << ((ring_ - a + nslots_) % nslots_);
    CRK_HIP(hipMemcpyAsync(s.valid, valid.data(), sizeof(uint32_t) * wd, hipMemcpyHostToDevice, st_));
    gcr_multidot(CRK_FORM_FP64, W, fcap, used_, wi, f, s.partial, s.valid, ci, st_);
  }
  // one pass over the ring: w^ = w - sum c_j W_j with its norm and <w^, r>
  // from the coefficients and the dots of the unmodified w (r is orthogonal to
  // every direction of its basis), normalised, and the residual update.  The
  // first step of the ring runs the same kernel with no stored direction, so
  // that an RHS's first step has the same bits whether or not it joins a ring
  // that other RHS already fill.
  const int64_t dn = rhs_dot_launch(CRK_FORM_FP64, wi, o.r.p, f.n, wd, f.rs, f.es, s.dpart, st_);
  gcr_gs_update_ring(CRK_FORM_FP64, W, fcap, used_ > 1 ? used_ : 0, used_ > 1 ? (ring_ + 1) % used_ : 0, wi, o.r.p,
                     ci, s.dpart, dn, s.active, s.breakdown, f, s.partial, s.rn2, s.hinv + size_t(ring_) * cap_,
                     s.ha + size_t(ring_) * cap_, st_);
  if (used_ > 1) CRK_HIP(hipStreamSynchronize(st_));  // valid lives on the host stack
  std::vector<double> rn2(wd);
  std::vector<int> bd(wd);
  CRK_HIP(hipMemcpyAsync(rn2.data(), s.rn2, sizeof(double) * wd, hipMemcpyDeviceToHost, st_));
  CRK_HIP(hipMemcpyAsync(bd.data(), s.breakdown, sizeof(int) * wd, hipMemcpyDeviceToHost, st_));
  CRK_HIP(hipStreamSynchronize(st_));
  bool need_true = false, update_x = false;
  // window[r] > 0: slot r's solution is brought up to date in this step, over
  // its cycle's directions up to the current one.  That happens exactly when
  // the slot itself needs x (a convergence claim or a restart, whose true
  // residual reads it, or a stop, which keeps it), so a slot's x is formed at
  // the same points of its recursion whatever other slots share the solve.
  std::vector<int> claim(wd, 0), restart(wd, 0), window(cap_, 0);
  for (int r = 0; r < wd; ++r) {
    if (state_[r] != kSlotRunning) continue;
    const int wr = nbasis_[r] + 1;
    iters_[r] += 1;
    if (bd[r]) {  // breakdown: keep the best x
      state_[r] = kSlotStopped;
      window[r] = wr;
      continue;
    }
    nbasis_[r] += 1;
    if (std::sqrt(rn2[r]) <= p_.tol * bn_[r]) { claim[r] = 1; need_true = true; window[r] = wr; }
    else if (nbasis_[r] >= nslots_) { restart[r] = 1; need_true = true; window[r] = wr; }
    if (iters_[r] >= p_.max_iter) window[r] = wr;
    update_x |= window[r] > 0;
  }
  if (update_x) materialize(wd, window, ring_);
  if (need_true) {
    true_residual(wd);
    std::vector<double> h3(3 * size_t(wd));
    CRK_HIP(hipMemcpyAsync(h3.data(), s.sums3, sizeof(double) * 3 * wd, hipMemcpyDeviceToHost, st_));
    CRK_HIP(hipStreamSynchronize(st_));
    std::vector<int> mask(wd, 0);
    for (int r = 0; r < wd; ++r) {
      if (claim[r]) {
        const double t = std::sqrt(h3[3 * r + 2]);
        if (t <= p_.tol * bn_[r]) { state_[r] = kSlotConverged; tres_[r] = t / bn_[r]; }
        else { mask[r] = 1; nbasis_[r] = 0; }
      } else if (restart[r]) {
        mask[r] = 1;
        nbasis_[r] = 0;
      }
    }
    CRK_HIP(hipMemcpyAsync(o.mask.p, mask.data(), sizeof(int) * wd, hipMemcpyHostToDevice, st_));
    field_masked_copy(CRK_FORM_FP64, o.tmp.p, o.r.p, o.mask.as<int>(), f, st_);
    CRK_HIP(hipStreamSynchronize(st_));
  }
  for (int r = 0; r < wd; ++r)
    if (state_[r] == kSlotRunning && iters_[r] >= p_.max_iter) state_[r] = kSlotStopped;
  const double t = wall_now();
  for (int r = 0; r < wd; ++r)
    if (was_running[r] && state_[r] != kSlotRunning) t_done_[r] = t;
  upload_active();
  ring_ = (ring_ + 1) % nslots_;
  return running();
}

void OuterSolver::materialize(int wd, const std::vector<int>& window, int last) {
  OuterWork& o = w_->ow;
  GcrScalars& s = o.s;
  const int64_t V = H_->V(0);
  CRK_HIP(hipMemcpyAsync(nbd_.p, window.data(), sizeof(int) * size_t(cap_), hipMemcpyHostToDevice, st_));
  gcr_ring_materialize(o.Z.p, o.z_form, 12 * V * cap_, nbd_.as<int>(), last, nslots_, cap_, o.x.p, s.hcoef, s.hinv,
                       s.ha, s.dcoef, fine_shape(V, wd), st_);
  CRK_HIP(hipStreamSynchronize(st_));  // window lives on the caller's stack
}

void OuterSolver::refresh_residuals() {
  // The solution of every slot that has stopped or converged is up to date
  // (step() forms it when a slot leaves the running state); a running slot's
  // value here is provisional and is formed again when it finishes.
  const int wd = width();
  if (wd == 0) return;
  true_residual(wd);
  std::vector<double> h3(3 * size_t(wd));
  CRK_HIP(hipMemcpyAsync(h3.data(), w_->ow.s.sums3, sizeof(double) * 3 * wd, hipMemcpyDeviceToHost, st_));
  CRK_HIP(hipStreamSynchronize(st_));
  for (int r = 0; r < wd; ++r)
    if (state_[r] != kSlotFree) tres_[r] = bn_[r] > 0 ? std::sqrt(h3[3 * r + 2]) / bn_[r] : 0.0;
}

void OuterSolver::export_x(int s0, int n, void* x_dev) {
  CRK_REQUIRE(n >= 1 && s0 >= 0 && s0 + n <= cap_, "slot range out of bounds");
  const int64_t V = H_->V(0);
  field_export(CRK_FORM_FP64, w_->ow.x.as<double2>() + 12 * V * s0, static_cast<double2*>(x_dev),
               H_->fine_geo.pos.as<int>(), V, 12, n, st_);
}

void OuterSolver::level_iters(int s0, int n, std::vector<std::vector<int>>& out) {
  out.assign(CRK_MAX_LEVELS, std::vector<int>(n, 0));
  for (int l = 1; l < H_->nlev && l < CRK_MAX_LEVELS; ++l)
    CRK_HIP(hipMemcpyAsync(out[l].data(), w_->lv[l].s.level_iters + s0, sizeof(int) * n, hipMemcpyDeviceToHost, st_));
  CRK_HIP(hipStreamSynchronize(st_));
  for (int i = 0; i < n; ++i) out[0][i] = iters_[s0 + i];
}

void OuterSolver::release(int s) {
  CRK_REQUIRE(s >= 0 && s < cap_, "slot out of bounds");
  if (state_[s] == kSlotFree) return;
  // A free slot inside the running width is still swept by the kernels: give it
  // a zero residual so that its inner solves stop at once.
  const int64_t per = 12 * H_->V(0);
  CRK_HIP(hipMemsetAsync(w_->ow.r.as<double2>() + per * s, 0, sizeof(double2) * size_t(per), st_));
  state_[s] = kSlotFree;
  upload_active();
}

// ------------------------------------------------------------------ entry points

Hierarchy::Hierarchy() = default;
Hierarchy::~Hierarchy() = default;

size_t mg_solve_footprint(Hierarchy* H, int nrhs, int form, const crk_solve_info& p) {
  const int64_t V0 = H->V(0);
  const int nslots = ring_slots(p);
  size_t b = sizeof(double2) * 12 * size_t(V0) * nrhs * (4 + size_t(nslots)) +
             vec_bytes(outer_z_form(H, form)) * 12 * size_t(V0) * nrhs * nslots;
  const int defer = post_defer(H->nlev, p);
  if (H->nlev > 1) b += (3 + size_t(defer > 1 ? defer : 0)) * vec_bytes(form) * 12 * size_t(V0) * nrhs;
  for (int l = 1; l < H->nlev; ++l) {
    const int maxit = l == H->nlev - 1 ? p.coarsest_maxit : p.inner_maxit;
    b += vec_bytes(form) * size_t(H->N(l)) * H->V(l) * nrhs * (5 + 2 * size_t(maxit));
  }
  return b;
}

int mg_solve_dev(Hierarchy* H, const void* b_dev, void* x_dev, int nrhs, hipStream_t st, crk_solve_info* info) {
  const crk_solve_info& p = *info;
  validate(H, p);
  CRK_REQUIRE(nrhs >= 1 && nrhs <= 64, "nrhs must be in [1, 64]");
  if (!H->ws || !workspace_fits(*H->ws, nrhs, p.form, p)) {
    H->ws.reset();
    H->ws = make_workspace(H, nrhs, p.form, p, st);
  }
  hipEvent_t t0, t1;
  CRK_HIP(hipEventCreate(&t0));
  CRK_HIP(hipEventCreate(&t1));
  CRK_HIP(hipEventRecord(t0, st));
  OuterSolver os(H, H->ws.get(), p, st);
  os.admit(0, nrhs, b_dev);
  while (os.step() > 0) {
  }
  os.refresh_residuals();  // final true residual of every RHS
  os.export_x(0, nrhs, x_dev);
  CRK_HIP(hipEventRecord(t1, st));
  std::vector<std::vector<int>> li;
  os.level_iters(0, nrhs, li);
  float ms = 0;
  CRK_HIP(hipEventElapsedTime(&ms, t0, t1));
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  info->seconds = ms * 1e-3;
  info->iters = 0;
  info->true_rel_resid = 0;
  for (int l = 0; l < CRK_MAX_LEVELS; ++l) info->level_iters[l] = 0;
  H->last_iters.assign(nrhs, 0);
  H->last_resid.assign(nrhs, 0);
  H->last_seconds.assign(nrhs, 0);
  bool all_conv = true;
  for (int r = 0; r < nrhs; ++r) {
    const double rr = os.true_rel(r);
    H->last_iters[r] = os.iters(r);
    H->last_resid[r] = rr;
    H->last_seconds[r] = os.seconds(r);
    info->iters = std::max(info->iters, os.iters(r));
    info->true_rel_resid = std::max(info->true_rel_resid, rr);
    all_conv &= rr <= p.tol;
    for (int l = 0; l < H->nlev && l < CRK_MAX_LEVELS; ++l)
      info->level_iters[l] = std::max(info->level_iters[l], li[l][r]);
  }
  return all_conv ? CRK_OK : CRK_ENOCONV;
}

}  // namespace crk
