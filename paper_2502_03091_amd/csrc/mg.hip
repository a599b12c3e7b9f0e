// Multigrid setup (paper, Sec. 2 Eq. (1), Sec. 3 Eqs. (2), (5), (6), Sec. 2 Eq. (4)).
//
// For every coarsening step l: MR smoother on D_l psi_i ~ 0 over m' vectors
// (one multi-RHS operator launch per sweep with the <Dr,r>, <Dr,Dr> partial
// sums fused into it), normalisation, chiral split + batched block SVD
// truncated to k per chirality (-> P, sigma), and the Galerkin coarse operator
// D_{l+1} = P^dag D_l P stored in FP64 with FP32 / FP16S copies.
#include "mg.h"
#include "clover.h"

#include <cmath>
#include <cstring>

#include "blas.h"
#include "coarse.h"
#include "galerkin.h"
#include "gcr.h"
#include "transfer.h"

namespace crk {

namespace {

struct EventTimer {
  hipEvent_t e[8];
  int n = 0;
  explicit EventTimer(int count) : n(count) {
    for (int i = 0; i < n; ++i) CRK_HIP(hipEventCreate(&e[i]));
  }
  ~EventTimer() {
    for (int i = 0; i < n; ++i) (void)hipEventDestroy(e[i]);
  }
  void mark(int i, hipStream_t st) { CRK_HIP(hipEventRecord(e[i], st)); }
  double sec(int a, int b) {
    float ms = 0;
    CRK_HIP(hipEventElapsedTime(&ms, e[a], e[b]));
    return ms * 1e-3;
  }
};

int64_t prod4(const int d[4]) { return int64_t(d[0]) * d[1] * d[2] * d[3]; }

void validate(const Lattice* L, const crk_mg_params& p) {
  CRK_REQUIRE(p.n_levels == 2 || p.n_levels == 3, "n_levels must be 2 or 3");
  CRK_REQUIRE(p.setup_form == CRK_FORM_FP64 || p.setup_form == CRK_FORM_FP32, "setup_form must be FP64 or FP32");
  CRK_REQUIRE(p.smooth_chunk >= 0 && p.svd_batch >= 0, "smooth_chunk and svd_batch must be >= 0");
  CRK_REQUIRE(p.coarse_init == 0 || p.coarse_init == 1, "coarse_init must be 0 or 1");
  CRK_REQUIRE(p.smooth_defer >= 0 && p.smooth_defer <= kMrMaxDefer, "smooth_defer must be in [0, 8]");
  static_assert(CRK_MAX_LEVELS == 3, "coarse_init restricts from the fine step only");
  for (int l = 1; p.coarse_init && l < p.n_levels - 1; ++l)
    CRK_REQUIRE(p.init_vectors[l] != nullptr || p.m_prime[l] <= p.m_prime[l - 1],
                "coarse_init: m' of a step must not exceed m' of the step before");
  CRK_REQUIRE(L->V % kVL == 0, "the fine lattice volume must be a multiple of 64 for a hierarchy");
  int dims[4];
  std::memcpy(dims, L->dims, sizeof(dims));
  int N = 12;
  for (int l = 0; l < p.n_levels - 1; ++l) {
    for (int mu = 0; mu < 4; ++mu) {
      CRK_REQUIRE(p.block[l][mu] >= 1, "block extents must be >= 1");
      CRK_REQUIRE(dims[mu] % p.block[l][mu] == 0,
                  "block extent " + std::to_string(p.block[l][mu]) + " does not divide lattice extent " +
                      std::to_string(dims[mu]) + " at level " + std::to_string(l));
    }
    const int nb = p.block[l][0] * p.block[l][1] * p.block[l][2] * p.block[l][3];
    const int nr = (N / 2) * nb;
    CRK_REQUIRE(p.m_prime[l] >= 1 && p.m_prime[l] <= 128, "m' must be in [1, 128]");
    CRK_REQUIRE(p.k[l] >= 8 && p.k[l] % 8 == 0 && p.k[l] <= 32,
                "k must be a multiple of 8 in [8, 32] (2k is the MFMA tile height)");
    CRK_REQUIRE(p.k[l] <= p.m_prime[l], "k must not exceed m'");
    CRK_REQUIRE(p.k[l] <= nr, "k must not exceed the block rows N_r = (N/2)*|block|");
    CRK_REQUIRE(p.n_smooth[l] >= 0, "n_smooth must be >= 0");
    for (int mu = 0; mu < 4; ++mu) dims[mu] /= p.block[l][mu];
    N = 2 * p.k[l];
  }
}

}  // namespace



// ------------------------------------------------------------------ level operators
void level_apply(Hierarchy* H, int l, int form, const void* in, void* out, int nrhs, hipStream_t st, double* partial,
                 bool negate, void* copy, int in_form) {
  if (l == 0) {
    CRK_REQUIRE(copy == nullptr, "the fine operator has no fused copy");
    Lattice* L = H->lat;
    WilsonArgs a{};
    a.form = form;
    a.in = in;
    a.out = out;
    a.gauge = H->fine_gauge[form].p;
    a.nbr = H->fine_geo.nbr.as<int>();
    a.V = H->fine_geo.V;
    a.nrhs = nrhs;
    a.diag = negate ? -L->diag() : L->diag();
    L->hw(a.hw);
    if (negate)
      for (double& h : a.hw) h = -h;
    a.partial = partial;
    a.rhs_per_thread = 4;
    a.clover = H->fine_clover[form].p;  // NULL without the clover term
    a.clover_sign = negate ? -1.0 : 1.0;
    const Geometry& g = H->fine_geo;
    a.tile4 = g.blocked && g.block[0] == 4 && g.block[1] == 4 && g.block[2] == 4 && g.block[3] == 4;
    a.in_form = in_form;
    wilson_apply(a, st);
  } else {
    CRK_REQUIRE(in_form < 0 || in_form == form, "coarse apply: input must be in the operator's form");
    const CoarseLevel& c = H->coarse[l - 1];
    CRK_REQUIRE(partial == nullptr, "coarse apply has no fused reduction");
    coarse_apply(form, c.N, c.links[form].p, in, out, c.geo.nbr.as<int>(), c.V, nrhs, negate, st, copy);
  }
}

void level_residual(Hierarchy* H, int l, int form, const void* in, const void* b, void* out, int nrhs,
                    hipStream_t st) {
  const Geometry& g = H->fine_geo;
  const bool tile4 = g.blocked && g.block[0] == 4 && g.block[1] == 4 && g.block[2] == 4 && g.block[3] == 4;
  if (l == 0 && form == CRK_FORM_FP32 && tile4 && H->fine_clover[form].p == nullptr) {
    // the FP32 tile operator forms b - D in in its store (one pass fewer over
    // the fine field than the operator followed by b - out)
    Lattice* L = H->lat;
    WilsonArgs a{};
    a.form = form;
    a.in = in;
    a.out = out;
    a.gauge = H->fine_gauge[form].p;
    a.nbr = g.nbr.as<int>();
    a.V = g.V;
    a.nrhs = nrhs;
    a.diag = L->diag();
    L->hw(a.hw);
    a.tile4 = 1;
    a.sub = b;
    wilson_apply(a, st);
    return;
  }
  level_apply(H, l, form, in, out, nrhs, st);
  const FieldShape f = l == 0 ? fine_shape(H->V(0), nrhs) : coarse_shape(H->V(l), H->N(l), nrhs);
  field_axpby_to(form == CRK_FORM_FP64 ? CRK_FORM_FP64 : CRK_FORM_FP32, out, b, out, -1.0, 1.0, f.total(), st);
}

static TransferGeom transfer_geom(Hierarchy* H, int l, int nrhs) {
  const Transfer& t = H->T[l];
  TransferGeom g{};
  g.h = t.h;
  g.nb = t.nb;
  g.k = t.k;
  g.nblocks = t.nblocks;
  const int64_t V = H->V(l);
  if (l == 0) { g.aosoa = 1; g.ncomp = 12; g.Vp = pad_sites(V); g.vr = g.vc = g.vs = 0; }
  else { g.aosoa = 0; g.ncomp = H->N(l); g.Vp = V; g.vr = 1; g.vc = nrhs; g.vs = int64_t(H->N(l)) * nrhs; }
  g.pos_c = H->coarse[l].geo.pos.as<int>();
  return g;
}

void level_restrict(Hierarchy* H, int l, int form, const void* fine, void* coarse, int nrhs, hipStream_t st) {
  const TransferGeom g = transfer_geom(H, l, nrhs);
  const bool d = form == CRK_FORM_FP64;
  transfer_restrict(d ? CRK_FORM_FP64 : CRK_FORM_FP32, g, d ? H->T[l].P64.p : H->T[l].P32.p, fine, coarse, nrhs, st);
}

void level_prolong(Hierarchy* H, int l, int form, const void* coarse, void* fine, int nrhs, bool add, hipStream_t st) {
  const TransferGeom g = transfer_geom(H, l, nrhs);
  const bool d = form == CRK_FORM_FP64;
  transfer_prolong(d ? CRK_FORM_FP64 : CRK_FORM_FP32, g, d ? H->T[l].P64.p : H->T[l].P32.p, coarse, fine, nrhs, add,
                   st);
}

// ------------------------------------------------------------------ setup
namespace {

// Convert a host complex128 [m][V][N] block (lexicographic sites) to the rhs-inner
// coarse layout [pos][N][m] on the device.
__global__ void coarse_import_kernel(const double2* __restrict__ src, void* dst, int dst_double,
                                     const int* __restrict__ pos, int64_t V, int N, int m) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= V * N * m) return;
  const int64_t r = i / (V * N), rem = i % (V * N), s = rem / N, c = rem % N;
  const int64_t p = pos ? pos[s] : s;
  const int64_t o = (p * N + c) * m + r;
  if (dst_double) static_cast<double2*>(dst)[o] = src[i];
  else static_cast<float2*>(dst)[o] = make_float2(float(src[i].x), float(src[i].y));
}

__global__ void coarse_export_kernel(const void* src, int src_double, double2* __restrict__ dst,
                                     const int* __restrict__ pos, int64_t V, int N, int m) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= V * N * m) return;
  const int64_t r = i / (V * N), rem = i % (V * N), s = rem / N, c = rem % N;
  const int64_t p = pos ? pos[s] : s;
  const int64_t o = (p * N + c) * m + r;
  if (src_double) dst[i] = static_cast<const double2*>(src)[o];
  else { const float2 v = static_cast<const float2*>(src)[o]; dst[i] = make_double2(v.x, v.y); }
}

void setup_step(Hierarchy* H, int l, hipStream_t st) {
  const crk_mg_params& p = H->params;
  Transfer& t = H->T[l];
  StageTiming& tm = H->timing[l];
  const int m = p.m_prime[l];
  const int form = p.setup_form;
  const int64_t V = H->V(l);
  const int N = H->N(l);
  const int64_t n = int64_t(N) * V;       // entries per vector
  const bool inner = l > 0;               // coarse fields are rhs-inner
  const size_t esz = form == CRK_FORM_FP64 ? sizeof(double2) : sizeof(float2);
  EventTimer ev(6);
  ev.mark(0, st);

  // ---- test vectors
  DevBuf& psi = H->vectors[l];
  psi.alloc(esz * n * m);
  H->vec_form[l] = form;
  if (p.init_vectors[l]) {
    DevBuf h(sizeof(double2) * n * m);
    CRK_HIP(hipMemcpyAsync(h.p, p.init_vectors[l], sizeof(double2) * n * m, hipMemcpyHostToDevice, st));
    if (!inner) {
      field_import(form, h.as<double2>(), psi.p, H->fine_geo.pos.as<int>(), V, 12, m, st);
    } else {
      hipLaunchKernelGGL(coarse_import_kernel, dim3(ceil_div(n * m, 256)), dim3(256), 0, st, h.as<double2>(), psi.p,
                         int(form == CRK_FORM_FP64), H->geo(l).pos.as<int>(), V, N, m);
      CRK_LAUNCH_CHECK();
    }
    CRK_HIP(hipStreamSynchronize(st));  // h is freed at scope exit
  } else if (inner && p.coarse_init) {
    // coarse test vectors Sigma_k V_k^dag of the previous step (Sec. 3, after
    // Eq. (5)), i.e. P^dag (psi_i / ||psi_i||), for its first m vectors.  Only the step from the fine level precedes a coarse
    // step (at most three levels); its vectors are rhs-outer, so the first m
    // are contiguous, and kept in the setup form both steps share.
    level_restrict(H, l - 1, form, H->vectors[l - 1].p, psi.p, m, st);
    scale_rhs_inner(form, psi.p, H->inv_norm[l - 1].as<double>(), n, m, st);
  } else {
    gaussian_fill(form, psi.p, n * m, p.seed, uint32_t(l), st);
  }

  // ---- MR smoother on D psi ~ 0:  r = -D psi; repeat q = D r, alpha, psi += alpha r, r -= alpha q
  // Every vector runs its own recursion, so on the fine level (rhs-outer
  // layout) the vectors may be smoothed in chunks: when the residual fields r
  // and q of all m' vectors would not fit comfortably next to them, the chunk
  // is halved until they do.
  int mc = m;
  if (!inner && p.smooth_chunk > 0) {
    mc = std::min(m, int(p.smooth_chunk));
  } else if (!inner) {
    const size_t fr = device_free_bytes();
    while (mc > 8 && 2 * esz * size_t(n) * size_t(mc) > fr / 10 * 6) mc = (mc + 1) / 2;
  }
  const int nchunk = (m + mc - 1) / mc;
  // Fine level: D sweeps share one pass over psi (mr_update_ring); the
  // residuals of the pending sweeps live in a ring of D + 1 fields.  Per
  // sweep this moves 4 fields plus 1/D of a field instead of 5.  The automatic
  // depth keeps the ring and q within 30 % of the free device memory.
  int D = 1;
  if (!inner && p.n_smooth[l] > 1) {
    if (p.smooth_defer > 0) {
      D = p.smooth_defer;
    } else {
      const size_t fr = device_free_bytes(), field = esz * size_t(n) * size_t(mc);
      for (int d : {8, 4, 2})
        if (size_t(d + 2) * field <= fr / 10 * 3) {
          D = d;
          break;
        }
    }
  }
  D = std::min(D, std::max(1, p.n_smooth[l]));  // a ring longer than the sweeps is never filled
  std::vector<DevBuf> ring(D == 1 ? 1 : D + 1);
  for (auto& b : ring) b.alloc(esz * n * mc);
  std::vector<void*> slots;
  for (auto& b : ring) slots.push_back(b.p);
  DevBuf q(esz * n * mc);
  const int64_t nsb = wilson_partial_blocks(V);
  const int64_t ndp = rhs_dot_partials(n, inner);
  DevBuf partial(sizeof(double) * 3 * mc * (nsb > ndp ? nsb : ndp));
  DevBuf sums(sizeof(double) * 3 * mc), alpha(sizeof(double2) * mc * D);
  // events around every fine operator launch; read once after the stage
  std::vector<hipEvent_t> dev_ev(inner ? 0 : 2 * size_t(p.n_smooth[l]) * nchunk);
  for (auto& e : dev_ev) CRK_HIP(hipEventCreate(&e));
  for (int ch = 0; ch < nchunk; ++ch) {
    const int c0 = ch * mc, mm = std::min(mc, m - c0);
    void* pc = static_cast<char*>(psi.p) + esz * size_t(n) * c0;  // rhs-outer: vectors c0 .. c0+mm-1
    const int64_t rs = inner ? 1 : n, es = inner ? mm : 1;
    MrSweeps mr(slots, alpha.as<double2>(), size_t(mc));
    level_apply(H, l, form, pc, mr.r(0), mm, st, nullptr, /*negate=*/true);
    for (int it = 0; it < p.n_smooth[l]; ++it) {
      void* rk = mr.r(it);
      double2* ak = mr.alpha(it);
      if (!inner) {
        hipEvent_t* e = dev_ev.data() + 2 * (size_t(ch) * p.n_smooth[l] + it);
        CRK_HIP(hipEventRecord(e[0], st));
        level_apply(H, l, form, rk, q.p, mm, st, partial.as<double>());
        CRK_HIP(hipEventRecord(e[1], st));
        reduce_partials(partial.as<double>(), nsb, mm, 3, sums.as<double>(), st);
      } else {
        level_apply(H, l, form, rk, q.p, mm, st);
        // sums = (<q, r>, <q, q>)
        rhs_dot(form, q.p, rk, n, mm, rs, es, partial.as<double>(), sums.as<double>(), st);
      }
      mr_alpha(sums.as<double>(), mm, ak, st);
      // the residual after the last sweep is not used: that update skips it
      mr.update(form, pc, q.p, it, p.n_smooth[l], n, mm, inner, st);
    }
  }
  ev.mark(1, st);
  double dsum = 0;
  if (!dev_ev.empty()) {
    CRK_HIP(hipEventSynchronize(dev_ev.back()));
    for (size_t i = 0; i < dev_ev.size(); i += 2) {
      float ms = 0;
      CRK_HIP(hipEventElapsedTime(&ms, dev_ev[i], dev_ev[i + 1]));
      dsum += ms * 1e-3;
    }
  }
  for (auto& e : dev_ev) (void)hipEventDestroy(e);
  // the smoother's residual fields are as large as the test vectors: give them
  // back before the SVD and Galerkin stages allocate P and the coarse links
  CRK_HIP(hipStreamSynchronize(st));
  ring.clear();
  q.release();
  const int launches = inner ? 0 : p.n_smooth[l] * nchunk;
  tm.dslash_count = launches;
  tm.dslash_avg = launches > 0 ? dsum / launches : 0;
  tm.smoother_chunk = mc;
  const int64_t rs = inner ? 1 : n, es = inner ? m : 1;

  // ---- normalisation factors 1/||psi_i||
  DevBuf& inv = H->inv_norm[l];
  inv.alloc(sizeof(double) * m);
  rhs_dot(form, psi.p, nullptr, n, m, rs, es, partial.as<double>(), sums.as<double>(), st);
  if (p.normalize) {
    inv_sqrt(sums.as<double>(), 3, 2, m, inv.as<double>(), st);
  } else {
    std::vector<double> ones(m, 1.0);
    CRK_HIP(hipMemcpyAsync(inv.p, ones.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
    CRK_HIP(hipStreamSynchronize(st));
  }

  // ---- chiral split + block SVD truncation -> P, sigma
  ChiralSrc src{};
  if (!inner) { src.aosoa = 1; src.ncomp = 12; src.Vp = pad_sites(V); src.si = src.sc = src.ss = 0; }
  else { src.aosoa = 0; src.ncomp = N; src.Vp = V; src.si = 1; src.sc = m; src.ss = int64_t(N) * m; }
  src.h = N / 2;
  src.nb = t.nb;
  src.m = m;
  src.nblocks = t.nblocks;
  // SVD work space (Gram matrices, rotations and B = A V per block): in
  // batches of blocks when all blocks at once would not fit in a quarter of
  // the free device memory, and at most kSvdWorkCap bytes at once (a few
  // thousand blocks already fill the device; allocating tens of GB for one
  // batch costs more than the kernels of the extra batches)
  int64_t wcap = t.nblocks;
  {
    constexpr size_t kSvdWorkCap = size_t(8) << 30;
    const size_t fr = device_free_bytes();
    const size_t per = svd_work_bytes(m, t.nr, 1);
    const int64_t fit = int64_t(std::min(fr / 4, kSvdWorkCap) / per);
    if (fit < wcap) wcap = std::max<int64_t>(1, fit);
    if (p.svd_batch > 0) wcap = std::min<int64_t>(t.nblocks, p.svd_batch);
  }
  DevBuf work(svd_work_bytes(m, t.nr, wcap));
  SvdWork w = svd_work_carve(work.p, m, t.nr, wcap);
  t.P64.alloc(sizeof(double2) * 2 * t.nblocks * t.k * t.nr);
  t.P32.alloc(sizeof(float2) * 2 * t.nblocks * t.k * t.nr);
  t.nsig = m < t.nr ? m : t.nr;
  t.sigma.alloc(sizeof(double) * 2 * t.nblocks * t.nsig);
  chiral_svd(src, form == CRK_FORM_FP64, psi.p, inv.as<double>(), t.k, w, wcap, t.P64.as<double2>(),
             t.sigma.as<double>(), st);
  field_convert(CRK_FORM_FP64, t.P64.p, CRK_FORM_FP32, t.P32.p, 2 * t.nblocks * t.k * t.nr, 1, 1, st);
  ev.mark(2, st);

  // ---- Galerkin coarse operator
  CoarseLevel& c = H->coarse[l];
  c.links[0].alloc(coarse_links_bytes(CRK_FORM_FP64, c.V, c.N));
  if (l == 0) {
    GalerkinArgs g{};
    g.P = t.P64.as<double2>();
    g.gauge = H->fine_gauge[0].as<double2>();
    g.nbr = H->fine_geo.nbr.as<int>();
    g.V = V;
    g.nb = t.nb;
    g.nr = t.nr;
    g.k = t.k;
    g.diag = H->lat->diag();
    g.clover = H->fine_clover[0].as<double2>();
    H->lat->hw(g.hw);
    g.ncoarse = t.nblocks;
    g.pos_c = c.geo.pos.as<int>();
    g.links = c.links[0].as<double2>();
    galerkin_fine(g, c.geo.nbr.as<int>(), c.V, st);
  } else {
    GalerkinCoarseArgs g{};
    g.P = t.P64.as<double2>();
    g.links = H->coarse[l - 1].links[0].as<double2>();
    g.nbr = H->coarse[l - 1].geo.nbr.as<int>();
    g.V = V;
    g.N = N;
    g.nb = t.nb;
    g.nr = t.nr;
    g.k = t.k;
    g.ncoarse = t.nblocks;
    g.pos_c = c.geo.pos.as<int>();
    g.out = c.links[0].as<double2>();
    galerkin_coarse(g, c.geo.nbr.as<int>(), c.V, st);
  }
  c.links[1].alloc(coarse_links_bytes(CRK_FORM_FP32, c.V, c.N));
  c.links[2].alloc(coarse_links_bytes(CRK_FORM_FP16S, c.V, c.N));
  coarse_links_convert(c.links[0].p, CRK_FORM_FP32, c.links[1].p, c.V, c.N, st);
  coarse_links_convert(c.links[0].p, CRK_FORM_FP16S, c.links[2].p, c.V, c.N, st);
  ev.mark(3, st);
  CRK_HIP(hipStreamSynchronize(st));
  tm.smoother = ev.sec(0, 1);
  tm.svd = ev.sec(1, 2);
  tm.galerkin = ev.sec(2, 3);
  tm.total = ev.sec(0, 3);
}

}  // namespace

Hierarchy* mg_setup(Lattice* L, const crk_mg_params& p) {
  CRK_REQUIRE_STATE(L->gauge_loaded, "gauge field not loaded");
  validate(L, p);
  auto H = std::make_unique<Hierarchy>();
  H->lat = L;
  L->refs++;
  try {
    H->params = p;
    H->nlev = p.n_levels;
    CRK_HIP(hipStreamCreateWithFlags(&H->stream, hipStreamNonBlocking));
    hipStream_t st = H->stream;
    H->fine_geo.build(L->dims, p.block[0], st);
    for (int f = 0; f < 3; ++f) {
      H->fine_gauge[f].alloc(gauge_bytes(f, L->V));
      gauge_convert(f, L->U64.as<double2>(), H->fine_gauge[f].p, H->fine_geo.pos.as<int>(), L->V, st);
      if (L->c_sw != 0.0) {  // the lattice's clover blocks in this hierarchy's site order
        H->fine_clover[f].alloc(clover_bytes(f, L->V));
        clover_convert(f, L->clover64.as<double2>(), H->fine_clover[f].p, H->fine_geo.pos.as<int>(), L->V, st);
      }
    }
    int dims[4];
    std::memcpy(dims, L->dims, sizeof(dims));
    int N = 12;
    H->coarse.resize(H->nlev - 1);
    H->T.resize(H->nlev - 1);
    H->vectors.resize(H->nlev - 1);
    H->inv_norm.resize(H->nlev - 1);
    H->vec_form.assign(H->nlev - 1, p.setup_form);
    H->timing.resize(H->nlev - 1);
    for (int l = 0; l < H->nlev - 1; ++l) {
      Transfer& t = H->T[l];
      std::memcpy(t.block, p.block[l], sizeof(t.block));
      t.nb = t.block[0] * t.block[1] * t.block[2] * t.block[3];
      t.h = N / 2;
      t.nr = t.h * t.nb;
      t.m = p.m_prime[l];
      t.k = p.k[l];
      int cd[4];
      for (int mu = 0; mu < 4; ++mu) cd[mu] = dims[mu] / t.block[mu];
      t.nblocks = prod4(cd);
      CoarseLevel& c = H->coarse[l];
      std::memcpy(c.dims, cd, sizeof(cd));
      c.V = t.nblocks;
      c.N = 2 * t.k;
      const bool further = l + 1 < H->nlev - 1;
      c.geo.build(cd, further ? p.block[l + 1] : nullptr, st);
      std::memcpy(dims, cd, sizeof(cd));
      N = c.N;
    }
    for (int l = 0; l < H->nlev - 1; ++l) setup_step(H.get(), l, st);
    CRK_HIP(hipStreamSynchronize(st));
  } catch (...) {
    Hierarchy* h = H.release();
    mg_destroy(h);
    throw;
  }
  return H.release();
}

void mg_destroy(Hierarchy* H) {
  if (!H) return;
  if (--H->refs > 0) return;
  if (H->stream) {
    (void)hipStreamSynchronize(H->stream);
    (void)hipStreamDestroy(H->stream);
  }
  Lattice* L = H->lat;
  delete H;
  lattice_release(L);
}

// ------------------------------------------------------------------ inspection helpers (used by the C ABI)
void mg_export_coarse(Hierarchy* H, int level, const void* src, int src_double, double2* dst_dev, int m,
                      hipStream_t st) {
  const int64_t V = H->V(level);
  const int N = H->N(level);
  hipLaunchKernelGGL(coarse_export_kernel, dim3(ceil_div(V * N * m, 256)), dim3(256), 0, st, src, src_double, dst_dev,
                     H->geo(level).pos.as<int>(), V, N, m);
  CRK_LAUNCH_CHECK();
}

void mg_import_coarse(Hierarchy* H, int level, const double2* src_dev, void* dst, int dst_double, int m,
                      hipStream_t st) {
  const int64_t V = H->V(level);
  const int N = H->N(level);
  hipLaunchKernelGGL(coarse_import_kernel, dim3(ceil_div(V * N * m, 256)), dim3(256), 0, st, src_dev, dst, dst_double,
                     H->geo(level).pos.as<int>(), V, N, m);
  CRK_LAUNCH_CHECK();
}

}  // namespace crk
