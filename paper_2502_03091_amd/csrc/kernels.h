// Host-side launch wrappers of the HIP kernels (all stream-ordered, no syncs).
#pragma once

#include "common.h"

namespace crk {

// ------------------------------------------------------------------ geometry
// Device position of every lexicographic site: block-major (block j, local l)
// -> j*|block| + l when block != nullptr, else identity.  Also the inverse map
// and the neighbour table in device positions, nbr[dir][pos], dir = 2mu (+), 2mu+1 (-).
void build_geometry(const int dims[4], const int* block, int* pos, int* inv, int* nbr, hipStream_t st);
// Block index and local index of every lexicographic site.
void build_block_map(const int dims[4], const int block[4], int* out_jl, hipStream_t st);

// Gauge: complex128 host layout [V][4][3][3] (device copy) -> form layout [mu][9][V] at device positions.
void gauge_convert(int form, const double2* src, void* dst, const int* pos, int64_t V, hipStream_t st);

// Fine fields: complex128 [nrhs][V][ncomp] (site lexicographic) <-> native [nrhs][ncomp][V] (device order).
void field_import(int form, const double2* src, void* dst, const int* pos, int64_t V, int ncomp, int nrhs,
                  hipStream_t st);
void field_export(int form, const void* src, double2* dst, const int* pos, int64_t V, int ncomp, int nrhs,
                  hipStream_t st);
// Native fine field precision conversion (same layout).
void field_convert(int src_form, const void* src, int dst_form, void* dst, int64_t V, int ncomp, int nrhs,
                   hipStream_t st);

// ------------------------------------------------------------------ Wilson dslash
struct WilsonArgs {
  int form;
  const void* in;
  void* out;
  const void* gauge;
  const int* nbr;
  int64_t V;
  int nrhs;
  double diag;      // m0 + sum_mu w_mu
  double hw[4];     // -w_mu / 2
  double* partial;  // optional [V/64][nrhs][3]: <Dr, r> (re, im), <Dr, Dr> per 64 sites
  int rhs_per_thread;
  int order = 0;    // 0: RHS groups of a site block consecutive; 1: site blocks of a RHS group consecutive
  int swizzle = 1;  // XCD-contiguous workgroup mapping
  int tile4 = 0;    // device order is block-major in 4^4 blocks (every extent a multiple of 4)
  // Wilson-clover: the site blocks diag 1 + C(x) in the form's storage (FP64
  // double2, else float2), site-vectorised [72][V] at device positions; they
  // replace the scalar diag.  clover_sign multiplies them (-1 for -D).
  const void* clover = nullptr;
  double clover_sign = 1.0;
  // Storage form of `in` when it is not `form`: only FP32 input to the FP64
  // operator (values widened exactly, FP64 arithmetic and output).  -1: `form`.
  int in_form = -1;
  // When set (FP32 on 4^4 blocks, no fused sums): out = sub - D in, sub a field
  // in the layout of out.  Other operators leave it to the caller (level_apply).
  const void* sub = nullptr;
};
void wilson_apply(const WilsonArgs& a, hipStream_t st);
int64_t wilson_partial_blocks(int64_t V);

}  // namespace crk
