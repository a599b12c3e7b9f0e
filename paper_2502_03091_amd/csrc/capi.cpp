// C ABI of the crk library: argument validation, error capture and dispatch.
#include <cmath>
#include <cstring>

#include "lattice.h"
#include "mg.h"

namespace {

thread_local std::string g_last_error;

template <class F> int guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const crk::Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return CRK_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return CRK_EINTERNAL;
  } catch (...) {
    g_last_error = "unknown exception";
    return CRK_EINTERNAL;
  }
}

}  // namespace

void crk_set_error_(const std::string& msg) { g_last_error = msg; }
void crk_clear_error_() { g_last_error.clear(); }

struct crk_lattice_s { crk::Lattice* L; };
struct crk_mg_s { crk::Hierarchy* H; };

using namespace crk;

namespace crk {

size_t lattice_dirac_stage_bytes(const Lattice* L, int form, int64_t nrhs) {
  auto up = [](size_t n) { return (n + 255) & ~size_t(255); };
  return up(sizeof(double2) * 12 * size_t(L->V) * size_t(nrhs)) + 2 * up(fine_field_bytes(form, L->V, nrhs));
}

}  // namespace crk

extern "C" {

int crk_version(void) { return 1 * 10000 + 0 * 100 + 0; }

const char* crk_last_error(void) { return g_last_error.c_str(); }

int crk_device_info(char* name, int32_t n, int64_t* hbm_bytes, int32_t* n_cu) {
  return guarded([&] {
    hipDeviceProp_t prop;
    CRK_HIP(hipGetDeviceProperties(&prop, 0));
    if (name && n > 0) {
      std::strncpy(name, prop.gcnArchName, size_t(n) - 1);
      name[n - 1] = 0;
    }
    if (hbm_bytes) *hbm_bytes = int64_t(prop.totalGlobalMem);
    if (n_cu) *n_cu = prop.multiProcessorCount;
    return CRK_OK;
  });
}

int crk_cached_memory_bytes(int64_t* bytes) {
  return guarded([&] {
    CRK_REQUIRE(bytes != nullptr, "bytes is NULL");
    int dev = 0;
    CRK_HIP(hipGetDevice(&dev));
    *bytes = int64_t(device_cached_bytes(dev));
    return CRK_OK;
  });
}

int crk_release_cached_memory(void) {
  return guarded([&] {
    device_release_cached();
    return CRK_OK;
  });
}

int crk_create_lattice(const int32_t dims[4], double m0, double xi, crk_lattice_t* out) {
  return guarded([&] {
    CRK_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    Lattice* L = lattice_create(dims, m0, xi);
    *out = new crk_lattice_s{L};
    return CRK_OK;
  });
}

int crk_lattice_set_clover(crk_lattice_t lat, double c_sw) {
  return guarded([&] {
    CRK_REQUIRE(lat && lat->L, "lattice handle is NULL");
    lattice_set_clover(lat->L, c_sw);
    return CRK_OK;
  });
}

int crk_load_gauge(crk_lattice_t lat, const double* U, int64_t n_doubles) {
  return guarded([&] {
    CRK_REQUIRE(lat && lat->L, "lattice handle is NULL");
    CRK_REQUIRE(n_doubles == 72 * lat->L->V, "gauge size must be 2*36*V doubles");
    lattice_load_gauge(lat->L, U);
    return CRK_OK;
  });
}

static void check_form(int form) {
  CRK_REQUIRE(form == CRK_FORM_FP64 || form == CRK_FORM_FP32 || form == CRK_FORM_FP16S, "unknown precision form");
}

static void dirac_native(Lattice* L, int form, const void* in, void* out, int nrhs, hipStream_t st) {
  WilsonArgs a{};
  a.form = form;
  a.in = in;
  a.out = out;
  a.gauge = L->gauge[form].p;
  a.nbr = L->geo.nbr.as<int>();
  a.V = L->V;
  a.nrhs = nrhs;
  a.diag = L->diag();
  L->hw(a.hw);
  a.partial = nullptr;
  a.rhs_per_thread = 4;
  a.clover = L->c_sw != 0.0 ? L->clover[form].p : nullptr;
  wilson_apply(a, st);
}

}  // extern "C"

namespace crk {

void lattice_dirac_apply_staged(Lattice* L, int form, const double* in, double* out, int nrhs, void* h, void* a,
                                void* b) {
  const size_t hb = sizeof(double2) * 12 * size_t(L->V) * nrhs;
  CRK_HIP(hipMemcpyAsync(h, in, hb, hipMemcpyHostToDevice, L->stream));
  field_import(form, static_cast<const double2*>(h), a, nullptr, L->V, 12, nrhs, L->stream);
  dirac_native(L, form, a, b, nrhs, L->stream);
  field_export(form, b, static_cast<double2*>(h), nullptr, L->V, 12, nrhs, L->stream);
  CRK_HIP(hipMemcpyAsync(out, h, hb, hipMemcpyDeviceToHost, L->stream));
  CRK_HIP(hipStreamSynchronize(L->stream));
}

}  // namespace crk

extern "C" {

int crk_dirac_apply(crk_lattice_t lat, int32_t form, const double* in, double* out, int32_t nrhs) {
  return guarded([&] {
    CRK_REQUIRE(lat && lat->L, "lattice handle is NULL");
    Lattice* L = lat->L;
    check_form(form);
    CRK_REQUIRE_STATE(L->gauge_loaded, "gauge field not loaded");
    CRK_REQUIRE(nrhs >= 0, "nrhs must be >= 0");
    CRK_REQUIRE(nrhs == 0 || (in && out), "NULL field pointer");
    if (nrhs == 0) return CRK_OK;
    const size_t hb = sizeof(double2) * 12 * size_t(L->V) * nrhs;
    DevBuf h(hb), a(fine_field_bytes(form, L->V, nrhs)), b(fine_field_bytes(form, L->V, nrhs));
    lattice_dirac_apply_staged(L, form, in, out, nrhs, h.p, a.p, b.p);
    return CRK_OK;
  });
}

int crk_dirac_apply_dev(crk_lattice_t lat, int32_t form, const void* in, void* out, int32_t nrhs, void* hip_stream) {
  return guarded([&] {
    CRK_REQUIRE(lat && lat->L, "lattice handle is NULL");
    check_form(form);
    CRK_REQUIRE_STATE(lat->L->gauge_loaded, "gauge field not loaded");
    CRK_REQUIRE(nrhs >= 0, "nrhs must be >= 0");
    if (nrhs == 0) return CRK_OK;
    CRK_REQUIRE(in && out, "NULL field pointer");
    dirac_native(lat->L, form, in, out, nrhs, static_cast<hipStream_t>(hip_stream));
    return CRK_OK;
  });
}

int64_t crk_field_bytes(crk_lattice_t lat, int32_t form, int32_t nrhs) {
  if (!lat || !lat->L || nrhs < 0 || form < 0 || form > 2) return -1;
  return int64_t(fine_field_bytes(form, lat->L->V, nrhs));
}

int crk_field_import_dev(crk_lattice_t lat, int32_t form, const void* src, void* dst, int32_t nrhs, void* hip_stream) {
  return guarded([&] {
    CRK_REQUIRE(lat && lat->L, "lattice handle is NULL");
    check_form(form);
    CRK_REQUIRE(nrhs >= 0, "nrhs must be >= 0");
    if (nrhs == 0) return CRK_OK;
    CRK_REQUIRE(src && dst, "NULL field pointer");
    field_import(form, static_cast<const double2*>(src), dst, nullptr, lat->L->V, 12, nrhs,
                 static_cast<hipStream_t>(hip_stream));
    return CRK_OK;
  });
}

int crk_field_export_dev(crk_lattice_t lat, int32_t form, const void* src, void* dst, int32_t nrhs, void* hip_stream) {
  return guarded([&] {
    CRK_REQUIRE(lat && lat->L, "lattice handle is NULL");
    check_form(form);
    CRK_REQUIRE(nrhs >= 0, "nrhs must be >= 0");
    if (nrhs == 0) return CRK_OK;
    CRK_REQUIRE(src && dst, "NULL field pointer");
    field_export(form, src, static_cast<double2*>(dst), nullptr, lat->L->V, 12, nrhs,
                 static_cast<hipStream_t>(hip_stream));
    return CRK_OK;
  });
}

int crk_lattice_get_map(crk_lattice_t lat, int32_t what, void* out, int64_t n_bytes) {
  return guarded([&] {
    CRK_REQUIRE(lat && lat->L, "lattice handle is NULL");
    CRK_REQUIRE(what == CRK_MAP_NEIGHBOR, "unknown map");
    Lattice* L = lat->L;
    CRK_REQUIRE(n_bytes == int64_t(sizeof(int)) * 8 * L->V, "n_bytes must be 4*8*V");
    CRK_REQUIRE(out != nullptr, "out is NULL");
    std::vector<int> t(size_t(8) * L->V);
    CRK_HIP(hipMemcpyAsync(t.data(), L->geo.nbr.p, sizeof(int) * 8 * L->V, hipMemcpyDeviceToHost, L->stream));
    CRK_HIP(hipStreamSynchronize(L->stream));
    int* o = static_cast<int*>(out);
    for (int64_t s = 0; s < L->V; ++s)
      for (int d = 0; d < 8; ++d) o[s * 8 + d] = t[size_t(d) * L->V + s];
    return CRK_OK;
  });
}

void crk_lattice_destroy(crk_lattice_t lat) {
  if (!lat) return;
  try { lattice_release(lat->L); } catch (...) {}
  delete lat;
}

}  // extern "C"
