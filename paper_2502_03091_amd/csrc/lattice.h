// Host-side lattice object: geometry, gauge storage in every precision form.
#pragma once

#include <atomic>
#include <vector>

#include "field.h"
#include "kernels.h"

namespace crk {

inline int64_t volume4(const int d[4]) { return int64_t(d[0]) * d[1] * d[2] * d[3]; }

// Geometry of one lattice in one site order (lexicographic or block-major).
struct Geometry {
  int dims[4] = {0, 0, 0, 0};
  int block[4] = {1, 1, 1, 1};
  bool blocked = false;
  int64_t V = 0;
  DevBuf pos, inv, nbr;  // int32 [V], [V], [8][V]

  void build(const int d[4], const int* b, hipStream_t st) {
    for (int mu = 0; mu < 4; ++mu) { dims[mu] = d[mu]; block[mu] = b ? b[mu] : 1; }
    blocked = b != nullptr;
    V = volume4(dims);
    pos.alloc(sizeof(int) * V);
    inv.alloc(sizeof(int) * V);
    nbr.alloc(sizeof(int) * 8 * V);
    build_geometry(dims, b, pos.as<int>(), inv.as<int>(), nbr.as<int>(), st);
  }
};

struct Lattice {
  int dims[4];
  int64_t V;
  double m0, xi;
  double w[4];
  Geometry geo;              // lexicographic
  DevBuf U64;                // complex128 host layout copy [V][4][3][3]
  DevBuf gauge[3];           // per form, [mu][9][V] lexicographic
  bool gauge_loaded = false;
  double c_sw = 0.0;         // clover coefficient (0: plain Wilson)
  DevBuf clover64;           // c_sw != 0: FP64 site blocks diag 1 + C(x), [V][72] lexicographic
  DevBuf clover[3];          // per form, site-vectorised [72][V] lexicographic
  hipStream_t stream = nullptr;
  int device = 0;            // HIP device current when the lattice was created
  std::atomic<int> refs{1};

  double diag() const { return m0 + w[0] + w[1] + w[2] + w[3]; }
  void hw(double out[4]) const { for (int mu = 0; mu < 4; ++mu) out[mu] = -0.5 * w[mu]; }
};

Lattice* lattice_create(const int32_t dims[4], double m0, double xi);
void lattice_load_gauge(Lattice* L, const double* U_host);
// Set the clover coefficient; recomputes the clover blocks when the gauge field is loaded.
void lattice_set_clover(Lattice* L, double c_sw);
void lattice_release(Lattice* L);

// D applied to nrhs host-layout fields (complex128 [nrhs][V][12], host memory)
// through device staging the caller provides: h holds the complex128 host
// layout, a and b the form's native layout (fine_field_bytes each).  Runs on
// the lattice's stream and waits for it.
void lattice_dirac_apply_staged(Lattice* L, int form, const double* in, double* out, int nrhs, void* h, void* a,
                                void* b);
// Bytes of the three staging buffers above, each rounded up to 256 bytes.
size_t lattice_dirac_stage_bytes(const Lattice* L, int form, int64_t nrhs);

}  // namespace crk
