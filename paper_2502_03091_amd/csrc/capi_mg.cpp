// C ABI of the multigrid hierarchy: setup, solve and inspection entry points.
#include <cmath>
#include <cstring>
#include <string>

#include "coarse.h"
#include "mg.h"
#include "server.h"

namespace crk {
void mg_export_coarse(Hierarchy* H, int level, const void* src, int src_double, double2* dst_dev, int m,
                      hipStream_t st);
void mg_import_coarse(Hierarchy* H, int level, const double2* src_dev, void* dst, int dst_double, int m,
                      hipStream_t st);
}  // namespace crk

struct crk_lattice_s { crk::Lattice* L; };
struct crk_mg_s { crk::Hierarchy* H; };
struct crk_server_s { crk::Server* S; };

using namespace crk;

namespace {

template <class F> int guarded_mg(F&& f) {
  try {
    return f();
  } catch (const crk::Error& e) {
    crk_set_error_(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    crk_set_error_("host allocation failed");
    return CRK_ENOMEM;
  } catch (const std::exception& e) {
    crk_set_error_(e.what());
    return CRK_EINTERNAL;
  } catch (...) {
    crk_set_error_("unknown exception");
    return CRK_EINTERNAL;
  }
}

Hierarchy* hier(crk_mg_t mg) {
  if (!mg || !mg->H) fail(CRK_EINVAL, "hierarchy handle is NULL");
  return mg->H;
}

void check_level(Hierarchy* H, int level, int lo, int hi) {
  CRK_REQUIRE(level >= lo && level <= hi, "level out of range");
  (void)H;
}

}  // namespace

extern "C" {

void crk_mg_params_default(crk_mg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->n_levels = 2;
  for (int l = 0; l < CRK_MAX_LEVELS; ++l) {
    p->m_prime[l] = 48;
    p->k[l] = 24;
    for (int mu = 0; mu < 4; ++mu) p->block[l][mu] = l == 0 ? 4 : 2;
    p->n_smooth[l] = 20;
  }
  p->setup_form = CRK_FORM_FP32;
  p->normalize = 1;
  p->seed = 0x2502030910ull;
}

int crk_mg_setup(crk_lattice_t lat, const crk_mg_params* params, crk_mg_t* out) {
  crk_clear_error_();
  return guarded_mg([&] {
    CRK_REQUIRE(lat && lat->L, "lattice handle is NULL");
    CRK_REQUIRE(params && out, "NULL argument");
    *out = nullptr;
    Hierarchy* H = mg_setup(lat->L, *params);
    // init vector pointers are the caller's; do not keep them
    for (int l = 0; l < CRK_MAX_LEVELS; ++l) H->params.init_vectors[l] = nullptr;
    *out = new crk_mg_s{H};
    return CRK_OK;
  });
}

void crk_solve_info_default(crk_solve_info* info) {
  if (!info) return;
  std::memset(info, 0, sizeof(*info));
  info->tol = 1e-10;
  info->max_iter = 200;
  info->form = CRK_FORM_FP64;
  info->restart = 16;
  info->tau = 0.1;
  info->inner_maxit = 20;
  info->coarsest_maxit = 50;
  info->nu_post = 4;
}

int crk_mg_solve_dev(crk_mg_t mg, const void* b_dev, void* x_dev, int32_t nrhs, void* hip_stream,
                     crk_solve_info* info) {
  crk_clear_error_();
  return guarded_mg([&] {
    Hierarchy* H = hier(mg);
    CRK_REQUIRE(info != nullptr, "info is NULL");
    CRK_REQUIRE(b_dev && x_dev, "NULL field pointer");
    const int rc = mg_solve_dev(H, b_dev, x_dev, nrhs, static_cast<hipStream_t>(hip_stream), info);
    if (rc == CRK_ENOCONV) crk_set_error_("solver did not reach the tolerance within max_iter");
    return rc;
  });
}

int crk_mg_solve(crk_mg_t mg, const double* b, double* x, int32_t nrhs, crk_solve_info* info) {
  crk_clear_error_();
  return guarded_mg([&] {
    Hierarchy* H = hier(mg);
    CRK_REQUIRE(info != nullptr, "info is NULL");
    CRK_REQUIRE(b && x, "NULL field pointer");
    CRK_REQUIRE(nrhs >= 1 && nrhs <= 64, "nrhs must be in [1, 64]");
    const size_t bytes = sizeof(double2) * 12 * size_t(H->V(0)) * nrhs;
    DevBuf db(bytes), dx(bytes);
    hipStream_t st = H->stream;
    CRK_HIP(hipMemcpyAsync(db.p, b, bytes, hipMemcpyHostToDevice, st));
    const int rc = mg_solve_dev(H, db.p, dx.p, nrhs, st, info);
    CRK_HIP(hipMemcpyAsync(x, dx.p, bytes, hipMemcpyDeviceToHost, st));
    CRK_HIP(hipStreamSynchronize(st));
    if (rc == CRK_ENOCONV) crk_set_error_("solver did not reach the tolerance within max_iter");
    return rc;
  });
}

int crk_mg_last_solve_rhs(crk_mg_t mg, int32_t* iters, double* resid, int32_t nrhs) {
  crk_clear_error_();
  return guarded_mg([&] {
    Hierarchy* H = hier(mg);
    CRK_REQUIRE(size_t(nrhs) == H->last_iters.size(), "nrhs does not match the last solve");
    for (int r = 0; r < nrhs; ++r) {
      if (iters) iters[r] = H->last_iters[r];
      if (resid) resid[r] = H->last_resid[r];
    }
    return CRK_OK;
  });
}

int crk_mg_last_solve_rhs_seconds(crk_mg_t mg, double* seconds, int32_t nrhs) {
  crk_clear_error_();
  return guarded_mg([&] {
    Hierarchy* H = hier(mg);
    CRK_REQUIRE(seconds != nullptr, "seconds is NULL");
    CRK_REQUIRE(size_t(nrhs) == H->last_seconds.size(), "nrhs does not match the last solve");
    for (int r = 0; r < nrhs; ++r) seconds[r] = H->last_seconds[r];
    return CRK_OK;
  });
}

int64_t crk_mg_get_bytes(crk_mg_t mg, int32_t level, int32_t what) {
  if (!mg || !mg->H) return -1;
  Hierarchy* H = mg->H;
  const int nstep = H->nlev - 1;
  if (what == CRK_GET_BLOCK_MAP || what == CRK_GET_DEVICE_ORDER) {
    if (level < 0 || level >= H->nlev) return -1;
    return int64_t(sizeof(int)) * H->V(level) * (what == CRK_GET_BLOCK_MAP ? 2 : 1);
  }
  if (level < 0 || level >= nstep) return -1;
  const Transfer& t = H->T[level];
  const CoarseLevel& c = H->coarse[level];
  switch (what) {
    case CRK_GET_P: return int64_t(sizeof(double2)) * 2 * t.nblocks * t.nr * t.k;
    case CRK_GET_SIGMA: return int64_t(sizeof(double)) * 2 * t.nblocks * t.nsig;
    case CRK_GET_X: return int64_t(sizeof(double2)) * c.V * c.N * c.N;
    case CRK_GET_YP:
    case CRK_GET_YM: return int64_t(sizeof(double2)) * 4 * c.V * c.N * c.N;
    case CRK_GET_VECTORS: return int64_t(sizeof(double2)) * t.m * H->V(level) * H->N(level);
    default: return -1;
  }
}

int crk_mg_get(crk_mg_t mg, int32_t level, int32_t what, void* out, int64_t n_bytes) {
  crk_clear_error_();
  return guarded_mg([&] {
    Hierarchy* H = hier(mg);
    const int64_t need = crk_mg_get_bytes(mg, level, what);
    CRK_REQUIRE(need >= 0, "unknown quantity or level");
    CRK_REQUIRE(n_bytes == need, "n_bytes must be " + std::to_string(need));
    CRK_REQUIRE(out != nullptr, "out is NULL");
    hipStream_t st = H->stream;
    if (what == CRK_GET_BLOCK_MAP) {
      CRK_REQUIRE(level < H->nlev - 1, "the coarsest level has no blocking");
      DevBuf d{size_t(need)};
      build_block_map(H->geo(level).dims, H->T[level].block, d.as<int>(), st);
      CRK_HIP(hipMemcpyAsync(out, d.p, size_t(need), hipMemcpyDeviceToHost, st));
      CRK_HIP(hipStreamSynchronize(st));
      return CRK_OK;
    }
    if (what == CRK_GET_DEVICE_ORDER) {
      CRK_HIP(hipMemcpyAsync(out, H->geo(level).pos.p, size_t(need), hipMemcpyDeviceToHost, st));
      CRK_HIP(hipStreamSynchronize(st));
      return CRK_OK;
    }
    const Transfer& t = H->T[level];
    const CoarseLevel& c = H->coarse[level];
    if (what == CRK_GET_P) {
      // device [pair][i][c'*nb + l]  ->  host [j][alpha][h*l + c'][i]
      std::vector<double2> d(size_t(2) * t.nblocks * t.k * t.nr);
      CRK_HIP(hipMemcpyAsync(d.data(), t.P64.p, sizeof(double2) * d.size(), hipMemcpyDeviceToHost, st));
      CRK_HIP(hipStreamSynchronize(st));
      double2* o = static_cast<double2*>(out);
      for (int64_t pr = 0; pr < 2 * t.nblocks; ++pr)
        for (int i = 0; i < t.k; ++i)
          for (int cp = 0; cp < t.h; ++cp)
            for (int l = 0; l < t.nb; ++l)
              o[(pr * t.nr + int64_t(t.h) * l + cp) * t.k + i] = d[(pr * t.k + i) * t.nr + int64_t(cp) * t.nb + l];
      return CRK_OK;
    }
    if (what == CRK_GET_SIGMA) {
      CRK_HIP(hipMemcpyAsync(out, t.sigma.p, size_t(need), hipMemcpyDeviceToHost, st));
      CRK_HIP(hipStreamSynchronize(st));
      return CRK_OK;
    }
    if (what == CRK_GET_X || what == CRK_GET_YP || what == CRK_GET_YM) {
      const int N = c.N;
      std::vector<double2> d(size_t(c.V) * 9 * N * N);
      std::vector<int> pos(c.V);
      CRK_HIP(hipMemcpyAsync(d.data(), c.links[0].p, sizeof(double2) * d.size(), hipMemcpyDeviceToHost, st));
      CRK_HIP(hipMemcpyAsync(pos.data(), c.geo.pos.p, sizeof(int) * c.V, hipMemcpyDeviceToHost, st));
      CRK_HIP(hipStreamSynchronize(st));
      double2* o = static_cast<double2*>(out);
      const int nmu = what == CRK_GET_X ? 1 : 4;
      for (int mu = 0; mu < nmu; ++mu) {
        const int nb = what == CRK_GET_X ? 0 : (what == CRK_GET_YP ? 1 + 2 * mu : 2 + 2 * mu);
        for (int64_t j = 0; j < c.V; ++j) {
          const double2* blk = d.data() + (int64_t(pos[j]) * 9 + nb) * N * N;
          double2* ob = o + (int64_t(mu) * c.V + j) * N * N;
          for (int r = 0; r < N; ++r)
            for (int cc = 0; cc < N; ++cc) ob[r * N + cc] = blk[cc * N + r];
        }
      }
      return CRK_OK;
    }
    if (what == CRK_GET_VECTORS) {
      const int m = t.m;
      const int64_t V = H->V(level);
      const int N = H->N(level);
      DevBuf tmp(sizeof(double2) * size_t(m) * V * N);
      if (level == 0)
        field_export(H->vec_form[0], H->vectors[0].p, tmp.as<double2>(), H->fine_geo.pos.as<int>(), V, 12, m, st);
      else
        mg_export_coarse(H, level, H->vectors[level].p, H->vec_form[level] == CRK_FORM_FP64, tmp.as<double2>(), m, st);
      std::vector<double> inv(m);
      CRK_HIP(hipMemcpyAsync(out, tmp.p, size_t(need), hipMemcpyDeviceToHost, st));
      CRK_HIP(hipMemcpyAsync(inv.data(), H->inv_norm[level].p, sizeof(double) * m, hipMemcpyDeviceToHost, st));
      CRK_HIP(hipStreamSynchronize(st));
      double* o = static_cast<double*>(out);
      const int64_t per = 2 * V * N;
      for (int i = 0; i < m; ++i)
        for (int64_t e = 0; e < per; ++e) o[i * per + e] *= inv[i];
      return CRK_OK;
    }
    fail(CRK_EINVAL, "unknown quantity");
  });
}

int crk_mg_get_timing(crk_mg_t mg, int32_t level, double* out6) {
  crk_clear_error_();
  return guarded_mg([&] {
    Hierarchy* H = hier(mg);
    CRK_REQUIRE(out6 != nullptr, "out is NULL");
    check_level(H, level, 0, H->nlev - 2);
    const StageTiming& t = H->timing[level];
    out6[0] = t.total;
    out6[1] = t.smoother;
    out6[2] = t.svd;
    out6[3] = t.galerkin;
    out6[4] = t.dslash_avg;
    out6[5] = t.dslash_count;
    return CRK_OK;
  });
}

// Fine vectors are FP32 for the FP16S form (the K-cycle's restriction and
// prolongation work on FP32 fields) unless fine_storage asks for the form's
// own storage (the fine operator of that form).
static void host_level_import(Hierarchy* H, int l, int form, const double* in, void* dst, int nrhs, hipStream_t st,
                              bool fine_storage = false) {
  const int64_t V = H->V(l);
  const int N = H->N(l);
  const size_t hb = sizeof(double2) * size_t(V) * N * nrhs;
  DevBuf h(hb);
  CRK_HIP(hipMemcpyAsync(h.p, in, hb, hipMemcpyHostToDevice, st));
  const int vf = form == CRK_FORM_FP64 ? CRK_FORM_FP64 : CRK_FORM_FP32;
  if (l == 0) field_import(fine_storage ? form : vf, h.as<double2>(), dst, H->fine_geo.pos.as<int>(), V, 12, nrhs, st);
  else mg_import_coarse(H, l, h.as<double2>(), dst, vf == CRK_FORM_FP64, nrhs, st);
  CRK_HIP(hipStreamSynchronize(st));
}

static void host_level_export(Hierarchy* H, int l, int form, const void* src, double* out, int nrhs, hipStream_t st,
                              bool fine_storage = false) {
  const int64_t V = H->V(l);
  const int N = H->N(l);
  const size_t hb = sizeof(double2) * size_t(V) * N * nrhs;
  DevBuf h(hb);
  const int vf = form == CRK_FORM_FP64 ? CRK_FORM_FP64 : CRK_FORM_FP32;
  if (l == 0) field_export(fine_storage ? form : vf, src, h.as<double2>(), H->fine_geo.pos.as<int>(), V, 12, nrhs, st);
  else mg_export_coarse(H, l, src, vf == CRK_FORM_FP64, h.as<double2>(), nrhs, st);
  CRK_HIP(hipMemcpyAsync(out, h.p, hb, hipMemcpyDeviceToHost, st));
  CRK_HIP(hipStreamSynchronize(st));
}

int crk_mg_coarse_apply(crk_mg_t mg, int32_t level, int32_t form, const double* in, double* out, int32_t nrhs) {
  crk_clear_error_();
  return guarded_mg([&] {
    Hierarchy* H = hier(mg);
    check_level(H, level, 0, H->nlev - 1);
    CRK_REQUIRE(form >= 0 && form <= 2, "unknown form");
    CRK_REQUIRE(nrhs >= 1 && in && out, "bad arguments");
    const size_t vb = level == 0 ? fine_field_bytes(form, H->V(0), nrhs)
                                 : (form == CRK_FORM_FP64 ? 16 : 8) * size_t(H->V(level)) * H->N(level) * nrhs;
    DevBuf a(vb), b(vb);
    hipStream_t st = H->stream;
    host_level_import(H, level, form, in, a.p, nrhs, st, true);
    level_apply(H, level, form, a.p, b.p, nrhs, st);
    host_level_export(H, level, form, b.p, out, nrhs, st, true);
    return CRK_OK;
  });
}

int64_t crk_mg_field_bytes(crk_mg_t mg, int32_t level, int32_t form, int32_t nrhs) {
  if (!mg || !mg->H || nrhs < 0 || form < 0 || form > 2) return -1;
  Hierarchy* H = mg->H;
  if (level < 0 || level >= H->nlev) return -1;
  if (level == 0) return int64_t(fine_field_bytes(form, H->V(0), nrhs));
  return int64_t(form == CRK_FORM_FP64 ? 16 : 8) * H->V(level) * H->N(level) * nrhs;
}

int crk_mg_apply_dev(crk_mg_t mg, int32_t level, int32_t form, const void* in, void* out, int32_t nrhs,
                     void* hip_stream) {
  crk_clear_error_();
  return guarded_mg([&] {
    Hierarchy* H = hier(mg);
    check_level(H, level, 0, H->nlev - 1);
    CRK_REQUIRE(form >= 0 && form <= 2, "unknown form");
    CRK_REQUIRE(nrhs >= 0, "nrhs must be >= 0");
    if (nrhs == 0) return CRK_OK;
    CRK_REQUIRE(in && out, "NULL field pointer");
    CRK_REQUIRE(in != out, "in and out must not alias");
    level_apply(H, level, form, in, out, nrhs, static_cast<hipStream_t>(hip_stream));
    return CRK_OK;
  });
}

int crk_mg_restrict(crk_mg_t mg, int32_t level, int32_t form, const double* in, double* out, int32_t nrhs) {
  crk_clear_error_();
  return guarded_mg([&] {
    Hierarchy* H = hier(mg);
    check_level(H, level, 0, H->nlev - 2);
    CRK_REQUIRE(form >= 0 && form <= 2, "unknown form");
    CRK_REQUIRE(nrhs >= 1 && in && out, "bad arguments");
    const size_t e = form == CRK_FORM_FP64 ? 16 : 8;
    DevBuf a(e * size_t(H->V(level)) * H->N(level) * nrhs), b(e * size_t(H->V(level + 1)) * H->N(level + 1) * nrhs);
    hipStream_t st = H->stream;
    host_level_import(H, level, form, in, a.p, nrhs, st);
    level_restrict(H, level, form, a.p, b.p, nrhs, st);
    host_level_export(H, level + 1, form, b.p, out, nrhs, st);
    return CRK_OK;
  });
}

int crk_mg_prolong(crk_mg_t mg, int32_t level, int32_t form, const double* in, double* out, int32_t nrhs) {
  crk_clear_error_();
  return guarded_mg([&] {
    Hierarchy* H = hier(mg);
    check_level(H, level, 0, H->nlev - 2);
    CRK_REQUIRE(form >= 0 && form <= 2, "unknown form");
    CRK_REQUIRE(nrhs >= 1 && in && out, "bad arguments");
    const size_t e = form == CRK_FORM_FP64 ? 16 : 8;
    DevBuf a(e * size_t(H->V(level + 1)) * H->N(level + 1) * nrhs), b(e * size_t(H->V(level)) * H->N(level) * nrhs);
    hipStream_t st = H->stream;
    host_level_import(H, level + 1, form, in, a.p, nrhs, st);
    level_prolong(H, level, form, a.p, b.p, nrhs, false, st);
    host_level_export(H, level, form, b.p, out, nrhs, st);
    return CRK_OK;
  });
}

int64_t crk_mg_footprint_bytes(crk_mg_t mg, int32_t nrhs, int32_t form) {
  if (!mg || !mg->H || nrhs < 1 || form < 0 || form > 2) return -1;
  Hierarchy* H = mg->H;
  size_t b = 0;
  b += H->fine_geo.pos.bytes + H->fine_geo.inv.bytes + H->fine_geo.nbr.bytes;
  for (int f = 0; f < 3; ++f) b += H->fine_gauge[f].bytes + H->fine_clover[f].bytes;
  for (auto& c : H->coarse) {
    b += c.geo.pos.bytes + c.geo.inv.bytes + c.geo.nbr.bytes;
    for (int f = 0; f < 3; ++f) b += c.links[f].bytes;
  }
  for (auto& t : H->T) b += t.P64.bytes + t.P32.bytes + t.sigma.bytes;
  for (auto& v : H->vectors) b += v.bytes;
  crk_solve_info p;
  crk_solve_info_default(&p);
  p.form = form;
  b += mg_solve_footprint(H, nrhs, form, p);
  return int64_t(b);
}

void crk_mg_destroy(crk_mg_t mg) {
  if (!mg) return;
  try { mg_destroy(mg->H); } catch (...) {}
  delete mg;
}


void crk_server_params_default(crk_server_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->hbm_budget_bytes = 0;
  p->slots_per_lane = 12;
  p->max_lanes = 4;
  p->idle_ms = 200;
  crk_solve_info_default(&p->solve);
  p->solve.form = CRK_FORM_FP32;
}

int crk_server_create(const crk_server_params* p, crk_server_t* out) {
  return guarded_mg([&] {
    crk_clear_error_();
    CRK_REQUIRE(p != nullptr && out != nullptr, "params and out must not be NULL");
    *out = nullptr;
    auto* h = new crk_server_s{nullptr};
    try {
      h->S = new Server(*p);
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
    return CRK_OK;
  });
}

int crk_server_add(crk_server_t srv, crk_mg_t mg, int32_t* lattice_id) {
  return guarded_mg([&] {
    crk_clear_error_();
    CRK_REQUIRE(srv && srv->S, "server handle is NULL");
    const int id = srv->S->add(hier(mg));
    if (lattice_id) *lattice_id = id;
    return CRK_OK;
  });
}

int crk_server_submit(crk_server_t srv, int32_t lattice_id, const double* b, double* x, int32_t nrhs,
                      uint64_t* request_id) {
  return guarded_mg([&] {
    crk_clear_error_();
    CRK_REQUIRE(srv && srv->S, "server handle is NULL");
    const uint64_t id = srv->S->submit(lattice_id, b, x, nrhs);
    if (request_id) *request_id = id;
    return CRK_OK;
  });
}

int crk_server_wait(crk_server_t srv, uint64_t request_id, double timeout_s, crk_request_info* info) {
  return guarded_mg([&] {
    crk_clear_error_();
    CRK_REQUIRE(srv && srv->S, "server handle is NULL");
    Request r;
    if (!srv->S->wait(request_id, timeout_s, r)) {
      crk_set_error_("request not finished within the timeout");
      return int(CRK_EBUSY);
    }
    if (info) {
      info->status = r.status;
      info->lattice = r.lattice;
      info->nrhs = r.nrhs;
      info->lane = r.lane;
      info->joined = r.joined ? 1 : 0;
      info->iters = r.iters;
      for (int l = 0; l < CRK_MAX_LEVELS; ++l) info->level_iters[l] = r.level_iters[l];
      info->true_rel_resid = r.resid;
      info->t_submit = r.t_submit;
      info->t_admit = r.t_admit;
      info->t_done = r.t_done;
    }
    if (r.status != CRK_OK) crk_set_error_(r.error);
    return r.status;
  });
}

int crk_server_get_stats(crk_server_t srv, crk_server_stats* out) {
  return guarded_mg([&] {
    crk_clear_error_();
    CRK_REQUIRE(srv && srv->S && out, "server handle or out is NULL");
    const ServerStats s = srv->S->stats();
    out->submitted = s.submitted;
    out->completed = s.completed;
    out->failed = s.failed;
    out->joins = s.joins;
    out->lanes_opened = s.lanes_opened;
    out->lanes_closed = s.lanes_closed;
    out->max_concurrent_lanes = s.max_concurrent_lanes;
    out->bytes_in_use = s.bytes_in_use;
    out->peak_bytes = s.peak_bytes;
    out->budget_bytes = int64_t(srv->S->budget());
    return CRK_OK;
  });
}

int64_t crk_server_lane_bytes(crk_server_t srv, int32_t lattice_id) {
  int64_t out = -1;
  const int rc = guarded_mg([&] {
    crk_clear_error_();
    CRK_REQUIRE(srv && srv->S, "server handle is NULL");
    out = int64_t(srv->S->lane_bytes(lattice_id));
    return CRK_OK;
  });
  return rc == CRK_OK ? out : rc;
}

void crk_server_destroy(crk_server_t srv) {
  if (!srv) return;
  try { delete srv->S; } catch (...) {}
  delete srv;
}

}  // extern "C"
