// Galerkin coarse operator of the fine Wilson level: interface.
#pragma once

#include "common.h"

namespace crk {

struct GalerkinArgs {
  const double2* P;      // [2*ncoarse][k][nr] prolongator blocks (row c'*nb + l)
  const double2* gauge;  // FP64 links [mu][9][V], fine device order (block-major)
  const int* nbr;        // fine neighbours [8][V], device positions
  int64_t V;
  int nb;                // fine sites per block
  int nr;                // 6*nb
  int k;
  double diag;           // m0 + sum w
  const double2* clover; // Wilson-clover: FP64 site blocks diag 1 + C(x), [72][V] site-vectorised at the
                         // fine device positions (NULL: plain Wilson, site term diag)
  double hw[4];          // -w_mu/2
  int64_t ncoarse;       // number of blocks (coarse sites)
  const int* pos_c;      // coarse device position of lexicographic coarse site (NULL = identity)
  double2* links;        // out: [Vc][9][2k][2k] column-major blocks, coarse device order
};

// Computes X and Y_{+mu}, then Y_{-mu} from sigma3-hermiticity using the
// coarse neighbour table nbr_c [8][Vc] (device positions).
void galerkin_fine(const GalerkinArgs& A, const int* nbr_c, int64_t Vc, hipStream_t st);

struct GalerkinCoarseArgs {
  const double2* P;      // [2*ncoarse][k][nr] prolongator blocks of this level (row c'*nb + l)
  const double2* links;  // this level's links [V][9][N][N] column-major, device order (block-major)
  const int* nbr;        // this level's neighbours [8][V]
  int64_t V;
  int N;                 // components per site on this level (2h)
  int nb, nr, k;         // sites per block, h*nb, kept vectors
  int64_t ncoarse;
  const int* pos_c;      // next level device position of lexicographic block j
  double2* out;          // next level links [Vc][9][2k][2k]
};

void galerkin_coarse(const GalerkinCoarseArgs& A, const int* nbr_c, int64_t Vc, hipStream_t st);

}  // namespace crk
