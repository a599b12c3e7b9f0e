// Lattice object: creation, gauge upload and conversion to every precision form.
#include "lattice.h"

#include "clover.h"

namespace crk {

Lattice* lattice_create(const int32_t dims[4], double m0, double xi) {
  CRK_REQUIRE(dims != nullptr, "dims is NULL");
  for (int mu = 0; mu < 4; ++mu) CRK_REQUIRE(dims[mu] >= 2, "every lattice extent must be >= 2");
  CRK_REQUIRE(xi > 0.0, "anisotropy xi must be > 0");
  CRK_REQUIRE(std::isfinite(m0), "m0 must be finite");
  const int64_t V = int64_t(dims[0]) * dims[1] * dims[2] * dims[3];
  CRK_REQUIRE(V <= (int64_t(1) << 30), "lattice volume above 2^30 sites is not supported");
  auto* L = new Lattice();
  try {
    for (int mu = 0; mu < 4; ++mu) L->dims[mu] = dims[mu];
    L->V = V;
    L->m0 = m0;
    L->xi = xi;
    L->w[0] = L->w[1] = L->w[2] = 1.0;
    L->w[3] = 1.0 / xi;
    CRK_HIP(hipGetDevice(&L->device));
    CRK_HIP(hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking));
    L->geo.build(L->dims, nullptr, L->stream);
    L->U64.alloc(sizeof(double2) * 36 * V);
    for (int f = 0; f < 3; ++f) L->gauge[f].alloc(gauge_bytes(f, V));
    CRK_HIP(hipStreamSynchronize(L->stream));
  } catch (...) {
    if (L->stream) (void)hipStreamDestroy(L->stream);
    delete L;
    throw;
  }
  return L;
}

void lattice_load_gauge(Lattice* L, const double* U_host) {
  CRK_REQUIRE(U_host != nullptr, "gauge pointer is NULL");
  CRK_HIP(hipMemcpyAsync(L->U64.p, U_host, sizeof(double2) * 36 * L->V, hipMemcpyHostToDevice, L->stream));
  for (int f = 0; f < 3; ++f)
    gauge_convert(f, L->U64.as<double2>(), L->gauge[f].p, L->geo.pos.as<int>(), L->V, L->stream);
  CRK_HIP(hipStreamSynchronize(L->stream));
  L->gauge_loaded = true;
  lattice_set_clover(L, L->c_sw);
}

void lattice_set_clover(Lattice* L, double c_sw) {
  CRK_REQUIRE(std::isfinite(c_sw), "c_sw must be finite");
  L->c_sw = c_sw;
  if (c_sw == 0.0) {
    L->clover64.release();
    for (int f = 0; f < 3; ++f) L->clover[f].release();
    return;
  }
  if (!L->gauge_loaded) return;  // computed when the gauge field arrives
  L->clover64.alloc(sizeof(double2) * 72 * size_t(L->V));
  clover_compute(L->U64.as<double2>(), L->dims, c_sw, L->w, L->diag(), L->clover64.as<double2>(), L->stream);
  for (int f = 0; f < 3; ++f) {
    L->clover[f].alloc(clover_bytes(f, L->V));
    clover_convert(f, L->clover64.as<double2>(), L->clover[f].p, L->geo.pos.as<int>(), L->V, L->stream);
  }
  CRK_HIP(hipStreamSynchronize(L->stream));
}

void lattice_release(Lattice* L) {
  if (!L) return;
  if (--L->refs == 0) {
    (void)hipStreamSynchronize(L->stream);
    (void)hipStreamDestroy(L->stream);
    delete L;
  }
}

}  // namespace crk
