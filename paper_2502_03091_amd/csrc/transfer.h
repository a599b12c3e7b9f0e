// Restriction / prolongation between consecutive levels: interface.
#pragma once

#include "common.h"

namespace crk {

struct TransferGeom {
  int h;              // components per chirality on the fine side of the step
  int nb;             // fine sites per block
  int k;              // kept vectors per chirality (coarse side has 2k components)
  int64_t nblocks;    // coarse sites
  int64_t vr, vc, vs; // fine-side strides (rhs, component, site) in complex entries
  int aosoa;          // 1: fine side is the site-vectorised fine layout (strides unused)
  int ncomp;          // components per fine site (aosoa)
  int64_t Vp;         // padded fine sites (aosoa)
  const int* pos_c;   // coarse device position of lexicographic block j (NULL = identity)
};

// coarse [Vc][2k][nrhs] = P^dag fine ; prec FP64 (double2, P64) or FP32 (float2, P32).
void transfer_restrict(int prec, const TransferGeom& g, const void* P, const void* fine, void* coarse, int nrhs,
                       hipStream_t st);
// fine (+)= P coarse.
void transfer_prolong(int prec, const TransferGeom& g, const void* P, const void* coarse, void* fine, int nrhs,
                      bool add, hipStream_t st);

}  // namespace crk
