// Multigrid hierarchy: levels, transfers, setup and solver entry points.
//
// Level 0 is the fine Wilson level (12 components per site); level l >= 1 is a
// Galerkin coarse stencil with N_l = 2 k_{l-1} components per site, chirality
// sigma_3 = first k vs last k components.  Every level stores its sites in the
// block-major order of the blocking that leads to the next level, so block
// operations read contiguous ranges; the coarsest level is lexicographic.
//
// Field layouts: level 0 is rhs-outer and site-vectorised (field.h); coarse
// levels are rhs-inner [V][N][nrhs] so that the MFMA coarse operator reads
// 16 right-hand sides of one component contiguously.
#pragma once

#include <atomic>
#include <map>
#include <memory>
#include <vector>

#include "lattice.h"
#include "svd.h"

namespace crk {

struct CoarseLevel {
  int dims[4] = {0, 0, 0, 0};
  int64_t V = 0;
  int N = 0;                 // components per site (2k of the previous step)
  Geometry geo;              // blocked if it is coarsened further
  DevBuf links[3];           // [V][9][N][N] column-major blocks per form (FP16S: half2 + scales)
};

struct Transfer {            // between level l and l+1
  int block[4] = {1, 1, 1, 1};
  int nb = 0;                // sites per block
  int h = 0;                 // components per chirality on level l
  int nr = 0;                // h * nb
  int m = 0, k = 0;
  int64_t nblocks = 0;       // = sites of level l+1
  int nsig = 0;
  DevBuf P64, P32;           // [2*nblocks][k][nr] complex
  DevBuf sigma;              // [2*nblocks][nsig]
};

struct StageTiming {
  double total = 0, smoother = 0, svd = 0, galerkin = 0, dslash_avg = 0, dslash_count = 0;
  int smoother_chunk = 0;  // vectors per smoother launch (all m' unless memory forced chunks)
};

struct Workspace;  // solver buffers (solver.cpp)

struct Hierarchy {
  Lattice* lat = nullptr;
  crk_mg_params params{};
  int nlev = 0;
  Geometry fine_geo;                 // block-major order of the fine lattice
  DevBuf fine_gauge[3];              // per form, fine device order
  DevBuf fine_clover[3];             // Wilson-clover: site blocks per form, fine device order (empty if c_sw = 0)
  std::vector<CoarseLevel> coarse;   // levels 1..nlev-1 (index l-1)
  std::vector<Transfer> T;           // steps 0..nlev-2
  std::vector<DevBuf> vectors;       // smoothed test vectors per step (setup form / coarse FP64)
  std::vector<DevBuf> inv_norm;      // per step [m]
  std::vector<int> vec_form;         // form of vectors[l]
  std::vector<StageTiming> timing;
  hipStream_t stream = nullptr;
  std::unique_ptr<Workspace> ws;
  std::vector<int> last_iters;
  std::vector<double> last_resid;
  std::vector<double> last_seconds;  // per RHS: admission to convergence (host wall time)
  std::atomic<int> refs{1};          // handle + every server that holds the hierarchy

  Hierarchy();
  ~Hierarchy();

  int64_t V(int l) const { return l == 0 ? fine_geo.V : coarse[l - 1].V; }
  int N(int l) const { return l == 0 ? 12 : coarse[l - 1].N; }
  const Geometry& geo(int l) const { return l == 0 ? fine_geo : coarse[l - 1].geo; }
};

Hierarchy* mg_setup(Lattice* L, const crk_mg_params& p);
void mg_destroy(Hierarchy* H);   // drops one reference; frees at zero

// Operators used by setup and solver (device fields in level layout, stream ordered).
// in_form >= 0: storage of `in` when it is not `form` (level 0 only: FP32 input to the FP64 operator).
void level_apply(Hierarchy* H, int l, int form, const void* in, void* out, int nrhs, hipStream_t st,
                 double* partial = nullptr, bool negate = false, void* copy = nullptr, int in_form = -1);
// out = b - D_l in (the residual of `in` for the right-hand sides b, in the level's layout).
void level_residual(Hierarchy* H, int l, int form, const void* in, const void* b, void* out, int nrhs,
                    hipStream_t st);
void level_restrict(Hierarchy* H, int l, int form, const void* fine, void* coarse, int nrhs, hipStream_t st);
void level_prolong(Hierarchy* H, int l, int form, const void* coarse, void* fine, int nrhs, bool add, hipStream_t st);

// Solve (solver.cpp).  b_dev/x_dev: complex128 host-layout device buffers [nrhs][V][12].
int mg_solve_dev(Hierarchy* H, const void* b_dev, void* x_dev, int nrhs, hipStream_t st, crk_solve_info* info);
size_t mg_solve_footprint(Hierarchy* H, int nrhs, int form, const crk_solve_info& p);

}  // namespace crk
