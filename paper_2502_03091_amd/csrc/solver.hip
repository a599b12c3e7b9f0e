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
#include <cmath>
#include <cstring>

#include "blas.h"
#include "coarse.h"
#include "gcr.h"
#include "mg.h"

namespace crk {

namespace {

// Device scalars of one GCR instance.
struct GcrScalars {
  DevBuf buf;
  double *sums3, *b2, *rn2, *inv, *partial;
  double2 *a, *coef;
  int *active, *iters, *breakdown, *n_active, *level_iters;
  uint32_t* valid;
  void alloc(int nrhs, int64_t partial_doubles) {
    const size_t nr = size_t(nrhs);
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off += (b + 255) & ~size_t(255); return o; };
    const size_t o_s3 = take(sizeof(double) * 3 * nr), o_b2 = take(sizeof(double) * nr),
                 o_rn = take(sizeof(double) * nr), o_inv = take(sizeof(double) * nr),
                 o_a = take(sizeof(double2) * nr), o_coef = take(sizeof(double2) * nr * kMaxCoef),
                 o_act = take(sizeof(int) * nr), o_it = take(sizeof(int) * nr), o_bd = take(sizeof(int) * nr),
                 o_na = take(sizeof(int)), o_li = take(sizeof(int) * nr), o_val = take(sizeof(uint32_t) * nr),
                 o_part = take(sizeof(double) * size_t(partial_doubles));
    buf.alloc(off);
    char* c = static_cast<char*>(buf.p);
    sums3 = reinterpret_cast<double*>(c + o_s3);
    b2 = reinterpret_cast<double*>(c + o_b2);
    rn2 = reinterpret_cast<double*>(c + o_rn);
    inv = reinterpret_cast<double*>(c + o_inv);
    a = reinterpret_cast<double2*>(c + o_a);
    coef = reinterpret_cast<double2*>(c + o_coef);
    active = reinterpret_cast<int*>(c + o_act);
    iters = reinterpret_cast<int*>(c + o_it);
    breakdown = reinterpret_cast<int*>(c + o_bd);
    n_active = reinterpret_cast<int*>(c + o_na);
    level_iters = reinterpret_cast<int*>(c + o_li);
    valid = reinterpret_cast<uint32_t*>(c + o_val);
    partial = reinterpret_cast<double*>(c + o_part);
  }
};

struct LevelWork {      // coarse level l >= 1: inner solve buffers (+ post-smoother fields)
  DevBuf x, r, b, Z, W, rho, q;
  int maxit = 0;
  GcrScalars s;
};

struct FineWork {       // level-0 K-cycle fields in the vector precision
  DevBuf rin, e, rho, q;
};

struct OuterWork {      // FP64 outer FGCR
  DevBuf b, x, r, tmp, Z, W;
  int nslots = 0;
  GcrScalars s;
};

constexpr int kPollEvery = 4;

int64_t partial_doubles(int64_t n, int nrhs) {
  const int64_t a = gcr_partial_rows(n) * nrhs * 2 * kMaxBasis;
  const int64_t b = rhs_dot_partials(n) * nrhs * 3;
  const int64_t c = wilson_partial_blocks(n / 12 + 1) * nrhs * 3;
  return std::max(a, std::max(b, c));
}

}  // namespace

struct Workspace {
  int nrhs = -1, form = -1, restart = -1, inner = -1, coarsest = -1;
  std::vector<LevelWork> lv;  // index l (0 unused)
  FineWork fw;
  OuterWork ow;
  size_t bytes = 0;
};

namespace {

int vec_prec(int form) { return form == CRK_FORM_FP64 ? CRK_FORM_FP64 : CRK_FORM_FP32; }
size_t vec_bytes(int form) { return form == CRK_FORM_FP64 ? sizeof(double2) : sizeof(float2); }
// Operator storage used on the fine level in a form (vectors there are FP32 for FP16S).
int fine_op_form(int form) { return form == CRK_FORM_FP64 ? CRK_FORM_FP64 : CRK_FORM_FP32; }

Workspace& workspace(Hierarchy* H, int nrhs, int form, const crk_solve_info& p) {
  if (!H->ws) H->ws = std::make_unique<Workspace>();
  Workspace& w = *H->ws;
  const int nslots = std::max(1, std::min(p.restart, p.max_iter));
  if (w.nrhs == nrhs && w.form == form && w.restart == nslots && w.inner == p.inner_maxit &&
      w.coarsest == p.coarsest_maxit)
    return w;
  w = Workspace();
  w.nrhs = nrhs;
  w.form = form;
  w.restart = nslots;
  w.inner = p.inner_maxit;
  w.coarsest = p.coarsest_maxit;
  const int64_t V0 = H->V(0);
  const size_t f64 = sizeof(double2) * 12 * size_t(V0) * nrhs;
  OuterWork& o = w.ow;
  o.nslots = nslots;
  o.b.alloc(f64); o.x.alloc(f64); o.r.alloc(f64); o.tmp.alloc(f64);
  o.Z.alloc(f64 * nslots); o.W.alloc(f64 * nslots);
  o.s.alloc(nrhs, partial_doubles(12 * V0, nrhs));
  w.bytes += f64 * (4 + 2 * size_t(nslots));
  if (H->nlev > 1) {
    const size_t fv = vec_bytes(form) * 12 * size_t(V0) * nrhs;
    w.fw.rin.alloc(fv); w.fw.e.alloc(fv); w.fw.rho.alloc(fv); w.fw.q.alloc(fv);
    w.bytes += 4 * fv;
  }
  w.lv.resize(H->nlev);
  for (int l = 1; l < H->nlev; ++l) {
    LevelWork& lw = w.lv[l];
    lw.maxit = l == H->nlev - 1 ? p.coarsest_maxit : p.inner_maxit;
    const size_t cv = vec_bytes(form) * size_t(H->N(l)) * H->V(l) * nrhs;
    lw.x.alloc(cv); lw.r.alloc(cv); lw.b.alloc(cv);
    if (l < H->nlev - 1) { lw.rho.alloc(cv); lw.q.alloc(cv); w.bytes += 2 * cv; }
    lw.Z.alloc(cv * lw.maxit); lw.W.alloc(cv * lw.maxit);
    lw.s.alloc(nrhs, partial_doubles(int64_t(H->N(l)) * H->V(l), nrhs));
    w.bytes += cv * (3 + 2 * size_t(lw.maxit));
  }
  return w;
}

FieldShape shape(Hierarchy* H, int l, int nrhs) {
  return l == 0 ? fine_shape(H->V(0), nrhs) : coarse_shape(H->V(l), H->N(l), nrhs);
}

void kcycle(Hierarchy* H, Workspace& w, int l, const crk_solve_info& p, const void* rin, void* eout, hipStream_t st);

// Inner flexible GCR on coarse level l: solves D_l x = b (lw.b) from x = 0.
void inner_fgcr(Hierarchy* H, Workspace& w, int l, const crk_solve_info& p, hipStream_t st) {
  LevelWork& lw = w.lv[l];
  const int nrhs = w.nrhs, form = w.form, prec = vec_prec(form);
  const FieldShape f = shape(H, l, nrhs);
  const int64_t fs = f.total();  // complex entries per stored field
  const size_t fb = vec_bytes(form) * size_t(fs);
  GcrScalars& s = lw.s;
  CRK_HIP(hipMemsetAsync(lw.x.p, 0, fb, st));
  CRK_HIP(hipMemcpyAsync(lw.r.p, lw.b.p, fb, hipMemcpyDeviceToDevice, st));
  rhs_dot(prec, lw.b.p, nullptr, f.n, nrhs, f.rs, f.es, s.partial, s.sums3, st);
  gcr_start(s.sums3, nrhs, s.b2, s.active, s.iters, s.n_active, st);
  const double tol2 = p.tau * p.tau;
  const bool precond = l < H->nlev - 1;
  char* Z = static_cast<char*>(lw.Z.p);
  char* W = static_cast<char*>(lw.W.p);
  int n_active = 1;
  for (int i = 0; i < lw.maxit; ++i) {
    void* zi = Z + fb * i;
    void* wi = W + fb * i;
    if (precond) kcycle(H, w, l, p, lw.r.p, zi, st);
    else CRK_HIP(hipMemcpyAsync(zi, lw.r.p, fb, hipMemcpyDeviceToDevice, st));
    level_apply(H, l, form, zi, wi, nrhs, st);
    if (i > 0) {
      gcr_multidot(prec, W, fs, i, wi, f, s.partial, nullptr, s.coef, st);
      gcr_multiaxpy(prec, Z, W, fs, i, zi, wi, s.coef, f, st);
    }
    rhs_dot(prec, wi, lw.r.p, f.n, nrhs, f.rs, f.es, s.partial, s.sums3, st);
    gcr_scalars(s.sums3, s.active, nrhs, s.inv, s.a, s.breakdown, st);
    gcr_update(prec, zi, wi, lw.x.p, lw.r.p, s.inv, s.a, s.active, f, s.partial, nullptr, st);
    gcr_check(s.partial, f, tol2, s.b2, s.breakdown, s.active, s.iters, s.rn2, s.n_active, s.level_iters, st);
    // Converged RHS are frozen on the device; the host only polls every few
    // iterations to stop launching once every RHS is done.
    if ((i + 1) % kPollEvery == 0 || i + 1 == lw.maxit) {
      CRK_HIP(hipMemcpyAsync(&n_active, s.n_active, sizeof(int), hipMemcpyDeviceToHost, st));
      CRK_HIP(hipStreamSynchronize(st));
      if (n_active == 0) break;
    }
  }
}

void kcycle(Hierarchy* H, Workspace& w, int l, const crk_solve_info& p, const void* rin, void* eout, hipStream_t st) {
  const int nrhs = w.nrhs, form = w.form, prec = vec_prec(form);
  const int opf = l == 0 ? fine_op_form(form) : form;
  LevelWork& nx = w.lv[l + 1];
  level_restrict(H, l, form, rin, nx.b.p, nrhs, st);
  inner_fgcr(H, w, l + 1, p, st);
  level_prolong(H, l, form, nx.x.p, eout, nrhs, false, st);
  if (p.nu_post <= 0) return;
  // MR on D_l e = r, starting from e:  rho = r - D e ; q = D rho ; e += alpha rho ; rho -= alpha q
  const FieldShape f = shape(H, l, nrhs);
  const size_t fb = vec_bytes(form) * size_t(f.total());
  void *rho, *q;
  if (l == 0) { rho = w.fw.rho.p; q = w.fw.q.p; }
  else { rho = w.lv[l].rho.p; q = w.lv[l].q.p; }
  GcrScalars& s = l == 0 ? w.ow.s : w.lv[l].s;
  // the scalars of level l are idle while its K-cycle runs (the cycle is called
  // between the solver's kernel phases); only sums3/partial/a are reused here.
  level_apply(H, l, opf, eout, q, nrhs, st);
  CRK_HIP(hipMemcpyAsync(rho, rin, fb, hipMemcpyDeviceToDevice, st));
  field_axpby(prec, q, rho, -1.0, 1.0, f.total(), st);
  for (int it = 0; it < p.nu_post; ++it) {
    if (l == 0) {
      level_apply(H, 0, opf, rho, q, nrhs, st, s.partial);
      reduce_partials(s.partial, wilson_partial_blocks(H->V(0)), nrhs, 3, s.sums3, st);
    } else {
      level_apply(H, l, opf, rho, q, nrhs, st);
      rhs_dot(prec, q, rho, f.n, nrhs, f.rs, f.es, s.partial, s.sums3, st);
    }
    mr_alpha(s.sums3, nrhs, s.a, st);
    mr_update(prec, eout, rho, q, s.a, f.n, nrhs, l > 0, st);
  }
}

}  // namespace

Hierarchy::Hierarchy() = default;
Hierarchy::~Hierarchy() = default;

size_t mg_solve_footprint(Hierarchy* H, int nrhs, int form, const crk_solve_info& p) {
  const int64_t V0 = H->V(0);
  const int nslots = std::max(1, std::min(p.restart, p.max_iter));
  size_t b = sizeof(double2) * 12 * size_t(V0) * nrhs * (4 + 2 * size_t(nslots));
  if (H->nlev > 1) b += 4 * vec_bytes(form) * 12 * size_t(V0) * nrhs;
  for (int l = 1; l < H->nlev; ++l) {
    const int maxit = l == H->nlev - 1 ? p.coarsest_maxit : p.inner_maxit;
    b += vec_bytes(form) * size_t(H->N(l)) * H->V(l) * nrhs * (5 + 2 * size_t(maxit));
  }
  return b;
}

int mg_solve_dev(Hierarchy* H, const void* b_dev, void* x_dev, int nrhs, hipStream_t st, crk_solve_info* info) {
  const crk_solve_info& p = *info;
  CRK_REQUIRE(p.tol > 0 && std::isfinite(p.tol), "tol must be > 0");
  CRK_REQUIRE(p.max_iter >= 1, "max_iter must be >= 1");
  CRK_REQUIRE(p.restart >= 1 && p.restart <= kMaxBasis, "restart must be in [1, 32]");
  CRK_REQUIRE(p.inner_maxit >= 1 && p.inner_maxit <= kMaxBasis, "inner_maxit must be in [1, 32]");
  CRK_REQUIRE(p.coarsest_maxit >= 1 && p.coarsest_maxit <= 64, "coarsest_maxit must be in [1, 64]");
  CRK_REQUIRE(p.form == CRK_FORM_FP64 || p.form == CRK_FORM_FP32 || p.form == CRK_FORM_FP16S, "unknown form");
  CRK_REQUIRE(p.tau > 0 && p.nu_post >= 0, "tau must be > 0 and nu_post >= 0");
  CRK_REQUIRE(nrhs >= 1 && nrhs <= 64, "nrhs must be in [1, 64]");
  Workspace& w = workspace(H, nrhs, p.form, p);
  // the coarsest GCR keeps up to coarsest_maxit directions
  CRK_REQUIRE(H->nlev == 1 || w.lv[H->nlev - 1].maxit <= 64, "coarsest basis too large");
  OuterWork& o = w.ow;
  GcrScalars& s = o.s;
  const int64_t V = H->V(0);
  const FieldShape f = fine_shape(V, nrhs);
  const int64_t fs = f.total();
  const size_t fb = sizeof(double2) * size_t(fs);
  const int* pos = H->fine_geo.pos.as<int>();
  hipEvent_t t0, t1;
  CRK_HIP(hipEventCreate(&t0));
  CRK_HIP(hipEventCreate(&t1));
  CRK_HIP(hipEventRecord(t0, st));

  // b (host layout, lexicographic) -> native FP64 block-major
  field_import(CRK_FORM_FP64, static_cast<const double2*>(b_dev), o.b.p, pos, V, 12, nrhs, st);
  CRK_HIP(hipMemsetAsync(o.x.p, 0, fb, st));
  CRK_HIP(hipMemcpyAsync(o.r.p, o.b.p, fb, hipMemcpyDeviceToDevice, st));
  for (int l = 1; l < H->nlev; ++l) CRK_HIP(hipMemsetAsync(w.lv[l].s.level_iters, 0, sizeof(int) * nrhs, st));
  rhs_dot(CRK_FORM_FP64, o.b.p, nullptr, f.n, nrhs, f.rs, f.es, s.partial, s.sums3, st);
  std::vector<double> h3(3 * size_t(nrhs));
  CRK_HIP(hipMemcpyAsync(h3.data(), s.sums3, sizeof(double) * 3 * nrhs, hipMemcpyDeviceToHost, st));
  CRK_HIP(hipStreamSynchronize(st));
  std::vector<double> bn(nrhs);
  std::vector<int> active(nrhs), iters(nrhs, 0), nbasis(nrhs, 0), conv(nrhs, 0), mask(nrhs, 0);
  std::vector<uint32_t> valid(nrhs, 0);
  std::vector<int> slot_of_age;  // unused placeholder for clarity
  for (int r = 0; r < nrhs; ++r) {
    bn[r] = std::sqrt(h3[3 * r + 2]);
    active[r] = bn[r] > 0;
    conv[r] = bn[r] == 0;
  }
  CRK_HIP(hipMemcpyAsync(s.active, active.data(), sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
  const int nslots = o.nslots;
  char* Z = static_cast<char*>(o.Z.p);
  char* W = static_cast<char*>(o.W.p);
  std::vector<double> rn2(nrhs), tn2(nrhs);
  int slot = 0, used = 0;
  for (int it = 0; it < p.max_iter; ++it) {
    bool any = false;
    for (int r = 0; r < nrhs; ++r) any |= active[r] != 0;
    if (!any) break;
    void* zi = Z + fb * slot;
    void* wi = W + fb * slot;
    if (H->nlev > 1) {
      void* rin = o.r.p;
      if (p.form != CRK_FORM_FP64) {
        field_convert(CRK_FORM_FP64, o.r.p, CRK_FORM_FP32, w.fw.rin.p, V, 12, nrhs, st);
        rin = w.fw.rin.p;
      }
      void* e = p.form == CRK_FORM_FP64 ? zi : w.fw.e.p;
      kcycle(H, w, 0, p, rin, e, st);
      if (p.form != CRK_FORM_FP64) field_convert(CRK_FORM_FP32, w.fw.e.p, CRK_FORM_FP64, zi, V, 12, nrhs, st);
    } else {
      CRK_HIP(hipMemcpyAsync(zi, o.r.p, fb, hipMemcpyDeviceToDevice, st));
    }
    level_apply(H, 0, CRK_FORM_FP64, zi, wi, nrhs, st);
    used = std::min(used + 1, nslots);
    if (used > 1) {
      for (int r = 0; r < nrhs; ++r) {
        uint32_t m = 0;
        for (int a = 1; a <= nbasis[r]; ++a) m |= 1u << ((slot - a + nslots) % nslots);
        valid[r] = m;
      }
      CRK_HIP(hipMemcpyAsync(s.valid, valid.data(), sizeof(uint32_t) * nrhs, hipMemcpyHostToDevice, st));
      gcr_multidot(CRK_FORM_FP64, W, fs, used, wi, f, s.partial, s.valid, s.coef, st);
      gcr_multiaxpy(CRK_FORM_FP64, Z, W, fs, used, zi, wi, s.coef, f, st);
    }
    rhs_dot(CRK_FORM_FP64, wi, o.r.p, f.n, nrhs, f.rs, f.es, s.partial, s.sums3, st);
    gcr_scalars(s.sums3, s.active, nrhs, s.inv, s.a, s.breakdown, st);
    gcr_update(CRK_FORM_FP64, zi, wi, o.x.p, o.r.p, s.inv, s.a, s.active, f, s.partial, s.rn2, st);
    std::vector<int> bd(nrhs);
    CRK_HIP(hipMemcpyAsync(rn2.data(), s.rn2, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    CRK_HIP(hipMemcpyAsync(bd.data(), s.breakdown, sizeof(int) * nrhs, hipMemcpyDeviceToHost, st));
    CRK_HIP(hipStreamSynchronize(st));
    bool need_true = false;
    std::vector<int> claim(nrhs, 0), restart(nrhs, 0);
    for (int r = 0; r < nrhs; ++r) {
      if (!active[r]) continue;
      iters[r] += 1;
      if (bd[r]) { active[r] = 0; continue; }  // breakdown: keep best x
      nbasis[r] += 1;
      if (std::sqrt(rn2[r]) <= p.tol * bn[r]) { claim[r] = 1; need_true = true; }
      else if (nbasis[r] >= nslots) { restart[r] = 1; need_true = true; }
    }
    if (need_true) {
      // tmp = b - D x  (true residual, FP64)
      level_apply(H, 0, CRK_FORM_FP64, o.x.p, o.tmp.p, nrhs, st);
      field_axpby(CRK_FORM_FP64, o.b.p, o.tmp.p, 1.0, -1.0, fs, st);
      rhs_dot(CRK_FORM_FP64, o.tmp.p, nullptr, f.n, nrhs, f.rs, f.es, s.partial, s.sums3, st);
      CRK_HIP(hipMemcpyAsync(h3.data(), s.sums3, sizeof(double) * 3 * nrhs, hipMemcpyDeviceToHost, st));
      CRK_HIP(hipStreamSynchronize(st));
      for (int r = 0; r < nrhs; ++r) {
        mask[r] = 0;
        if (claim[r]) {
          if (std::sqrt(h3[3 * r + 2]) <= p.tol * bn[r]) { conv[r] = 1; active[r] = 0; }
          else { mask[r] = 1; nbasis[r] = 0; }
        } else if (restart[r]) {
          mask[r] = 1;
          nbasis[r] = 0;
        }
      }
      DevBuf dm(sizeof(int) * nrhs);
      CRK_HIP(hipMemcpyAsync(dm.p, mask.data(), sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
      field_masked_copy(CRK_FORM_FP64, o.tmp.p, o.r.p, dm.as<int>(), f, st);
      CRK_HIP(hipMemcpyAsync(s.active, active.data(), sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
      CRK_HIP(hipStreamSynchronize(st));
    } else {
      CRK_HIP(hipMemcpyAsync(s.active, active.data(), sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
    }
    slot = (slot + 1) % nslots;
  }
  // final true residual of every RHS
  level_apply(H, 0, CRK_FORM_FP64, o.x.p, o.tmp.p, nrhs, st);
  field_axpby(CRK_FORM_FP64, o.b.p, o.tmp.p, 1.0, -1.0, fs, st);
  rhs_dot(CRK_FORM_FP64, o.tmp.p, nullptr, f.n, nrhs, f.rs, f.es, s.partial, s.sums3, st);
  field_export(CRK_FORM_FP64, o.x.p, static_cast<double2*>(x_dev), pos, V, 12, nrhs, st);
  CRK_HIP(hipEventRecord(t1, st));
  CRK_HIP(hipMemcpyAsync(h3.data(), s.sums3, sizeof(double) * 3 * nrhs, hipMemcpyDeviceToHost, st));
  std::vector<std::vector<int>> li(H->nlev);
  for (int l = 1; l < H->nlev; ++l) {
    li[l].resize(nrhs);
    CRK_HIP(hipMemcpyAsync(li[l].data(), w.lv[l].s.level_iters, sizeof(int) * nrhs, hipMemcpyDeviceToHost, st));
  }
  CRK_HIP(hipStreamSynchronize(st));
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
  bool all_conv = true;
  for (int r = 0; r < nrhs; ++r) {
    const double rr = bn[r] > 0 ? std::sqrt(h3[3 * r + 2]) / bn[r] : 0.0;
    H->last_iters[r] = iters[r];
    H->last_resid[r] = rr;
    info->iters = std::max(info->iters, iters[r]);
    info->true_rel_resid = std::max(info->true_rel_resid, rr);
    all_conv &= rr <= p.tol;
    info->level_iters[0] = std::max(info->level_iters[0], iters[r]);
    for (int l = 1; l < H->nlev && l < CRK_MAX_LEVELS; ++l) info->level_iters[l] = std::max(info->level_iters[l], li[l][r]);
  }
  return all_conv ? CRK_OK : CRK_ENOCONV;
}

}  // namespace crk
