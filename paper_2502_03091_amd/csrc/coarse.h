// Coarse stencil operator on MFMA: interface.
#pragma once

#include "common.h"

namespace crk {

// Bytes of the coarse links of Vc sites with N components in a form
// (FP16S: half2 blocks followed by one float scale per (site, link)).
size_t coarse_links_bytes(int form, int64_t Vc, int N);

// FP64 links [Vc][9][N][N] -> FP32 or FP16S copy.
void coarse_links_convert(const void* links64, int form, void* dst, int64_t Vc, int N, hipStream_t st);

// out = (negate ? -1 : 1) * D_c in; fields rhs-inner [Vc][N][nrhs] complex (double2 for FP64,
// float2 for FP32 and FP16S); nbr [8][Vc] device positions; N in {16, 32, 48, 64}.
// copy (optional, same layout): receives a copy of in in the same launch.
void coarse_apply(int form, int N, const void* links, const void* in, void* out, const int* nbr, int64_t Vc, int nrhs,
                  bool negate, hipStream_t st, void* copy = nullptr);

}  // namespace crk
