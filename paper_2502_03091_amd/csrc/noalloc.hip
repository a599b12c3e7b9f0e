// crk_dirac_apply_noalloc: the Wilson-Dirac operator on host buffers with no
// device allocation.
//
// crk_dirac_apply stages its host input and output through three device
// buffers it allocates per call (the complex128 host layout and the form's
// native input and output layouts).  This variant stages through one
// file-scope device array of fixed size instead, so it calls no hipMalloc,
// hipFree or allocating library routine.  Each GPU holds its own copy of the
// array for the life of the process; its address on a device is looked up
// once, with that device current, and kept per device.  Every call on one GPU
// shares that GPU's array: calls that overlap on one GPU (two host threads)
// race on it.  Every byte a call reads from the array is written by the same
// call first (the import writes every real site, the operator reads and
// writes real sites only, the export reads real sites only), so nothing needs
// clearing between calls.
#include <mutex>

#include "lattice.h"

struct crk_lattice_s { crk::Lattice* L; };

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of the scratch array (looked up once per device).
void* scratch_on(int device) {
  CRK_REQUIRE(device >= 0 && device < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch_ptr[device]) return g_scratch_ptr[device];
  int cur = 0;
  CRK_HIP(hipGetDevice(&cur));
  if (cur != device) CRK_HIP(hipSetDevice(device));
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) CRK_HIP(hipSetDevice(cur));
  CRK_HIP(e);
  CRK_REQUIRE(p != nullptr, "hipGetSymbolAddress returned NULL for the scratch array");
  g_scratch_ptr[device] = p;
  return p;
}

}  // namespace

extern "C" {

int64_t crk_dirac_apply_noalloc_max_bytes(void) { return int64_t(kScratchBytes); }

int crk_dirac_apply_noalloc(crk_lattice_t lat, int32_t form, const double* in, double* out, int32_t nrhs) {
  using namespace crk;
  crk_clear_error_();
  try {
    CRK_REQUIRE(lat && lat->L, "lattice handle is NULL");
    Lattice* L = lat->L;
    CRK_REQUIRE(form == CRK_FORM_FP64 || form == CRK_FORM_FP32 || form == CRK_FORM_FP16S, "unknown precision form");
    CRK_REQUIRE_STATE(L->gauge_loaded, "gauge field not loaded");
    CRK_REQUIRE(nrhs >= 0, "nrhs must be >= 0");
    CRK_REQUIRE(nrhs == 0 || (in && out), "NULL field pointer");
    if (nrhs == 0) return CRK_OK;
    const size_t need = lattice_dirac_stage_bytes(L, form, nrhs);
    CRK_REQUIRE(need <= kScratchBytes,
                "crk_dirac_apply_noalloc: " + std::to_string(need) + " bytes of staging exceed the fixed " +
                    std::to_string(kScratchBytes) + "-byte scratch array (fewer right-hand sides per call, or "
                    "crk_dirac_apply)");
    auto* base = static_cast<unsigned char*>(scratch_on(L->device));
    auto up = [](size_t n) { return (n + 255) & ~size_t(255); };
    const size_t hb = up(sizeof(double2) * 12 * size_t(L->V) * size_t(nrhs));
    const size_t fb = up(fine_field_bytes(form, L->V, nrhs));
    lattice_dirac_apply_staged(L, form, in, out, nrhs, base, base + hb, base + hb + fb);
    return CRK_OK;
  } catch (const Error& e) {
    crk_set_error_(e.what());
    return e.code;
  } catch (const std::exception& e) {
    crk_set_error_(e.what());
    return CRK_EINTERNAL;
  } catch (...) {
    crk_set_error_("unknown exception");
    return CRK_EINTERNAL;
  }
}

}  // extern "C"
