// Clover site term of the Wilson-clover operator: interface.
#pragma once

#include "common.h"

namespace crk {

// FP64 site blocks X(x) = diag 1 + C(x) of every lexicographic site, [V][72]
// complex128 (entry 36*alpha + 6*r + c: row r, column c of chirality alpha's
// 6 x 6 block), from the FP64 gauge field in host layout [V][4][3][3].
// Blocks until done (it frees its field-strength work space).
void clover_compute(const double2* U, const int dims[4], double c_sw, const double w[4], double diag, double2* X,
                    hipStream_t st);

// X in the site-vectorised layout of a form (72 components, FP64 double2,
// FP32 / FP16S float2), site x at device position pos[x] (NULL: identity).
void clover_convert(int form, const double2* X, void* dst, const int* pos, int64_t V, hipStream_t st);
size_t clover_bytes(int form, int64_t V);

}  // namespace crk
