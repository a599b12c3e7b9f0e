// Batched chiral SVD truncation: interface.
#pragma once

#include "common.h"

namespace crk {

// Where block matrix A_{j,alpha} lives: element (column i, component c, site)
// at base[i*si + c*sc + site*ss]; block j covers sites [j*nb, (j+1)*nb) of the
// device order; chirality alpha takes components [alpha*h, (alpha+1)*h).
struct ChiralSrc {
  int64_t si, sc, ss;
  int aosoa;    // 1: site-vectorised fine layout (entries at aidx(i, c, site, Vp, ncomp)), strides unused
  int ncomp;
  int64_t Vp;
  int h;        // components per chirality (6 fine, k coarse)
  int nb;       // sites per block
  int m;        // columns (test vectors)
  int64_t nblocks;
  int64_t j0 = 0;  // first block of the batch the kernels process (set by chiral_svd)
};

struct SvdWork {
  double2 *G, *V, *G2, *W, *B;
  double *lam, *lam2;
  int* sweeps;
  // m' > 64 only: packed Gram matrix, eigenvectors being accumulated (mm x mm),
  // recorded rotations of one Jacobi segment, per-matrix segment state
  double2 *Gp, *Vg;
  void* rec;
  int* state;
};

size_t svd_work_bytes(int m, int nr, int64_t nblocks);
SvdWork svd_work_carve(void* p, int m, int nr, int64_t nblocks);

// P: [2*nblocks][k][N_r] complex128 (pair = 2j + alpha, row rho = c'*nb + l);
// sigma: [2*nblocks][min(m, N_r)].  inv_norm (optional): per-column scale.
// w holds work space for wcap blocks; the blocks are processed in batches of wcap.
void chiral_svd(const ChiralSrc& s, int src_is_double, const void* base, const double* inv_norm, int k,
                const SvdWork& w, int64_t wcap, double2* P, double* sigma, hipStream_t st);

}  // namespace crk
