// Precision forms and native device field layouts.
//
// Fine-level fields of nrhs right-hand sides are stored component-major and
// site-fastest: element (r, c, s) at index (r*12 + c)*V + s, complex
// interleaved.  A wavefront therefore reads 64 consecutive sites of one
// component in one coalesced access.  FP16S stores half2 values of x/scale
// with one fp32 scale per (r, s), the largest |re|,|im| of that site's 24 reals.
#pragma once

#include "common.h"

namespace crk {

template <int FORM> struct Prec;
template <> struct Prec<CRK_FORM_FP64> { using real = double; using cx = double2; using store = double2; };
template <> struct Prec<CRK_FORM_FP32> { using real = float; using cx = float2; using store = float2; };
template <> struct Prec<CRK_FORM_FP16S> { using real = float; using cx = float2; using store = __half2; };

inline size_t store_bytes(int form) { return form == CRK_FORM_FP64 ? 16 : form == CRK_FORM_FP32 ? 8 : 4; }

// Bytes of a fine field set: data plus (FP16S) scales.
inline size_t fine_field_bytes(int form, int64_t V, int64_t nrhs, int ncomp = 12) {
  size_t b = store_bytes(form) * size_t(nrhs) * size_t(ncomp) * size_t(V);
  if (form == CRK_FORM_FP16S) b += sizeof(float) * size_t(nrhs) * size_t(V);
  return b;
}

template <int FORM> struct FineView {
  using S = typename Prec<FORM>::store;
  using C = typename Prec<FORM>::cx;
  S* data;
  float* scale;  // FP16S only: [nrhs][V]
  int64_t V;

  __host__ __device__ FineView() : data(nullptr), scale(nullptr), V(0) {}
  __host__ FineView(void* base, int64_t V_, int64_t nrhs) : data(static_cast<S*>(base)), scale(nullptr), V(V_) {
    if (FORM == CRK_FORM_FP16S)
      scale = reinterpret_cast<float*>(static_cast<char*>(base) + sizeof(S) * size_t(nrhs) * 12 * size_t(V_));
  }

  __device__ __forceinline__ void load(int64_t r, int64_t s, C v[12]) const {
    const S* p = data + r * 12 * V + s;
    if constexpr (FORM == CRK_FORM_FP16S) {
      float sc = scale[r * V + s];
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        float2 f = __half22float2(p[c * V]);
        v[c] = mk<float2>(f.x * sc, f.y * sc);
      }
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) v[c] = p[c * V];
    }
  }

  __device__ __forceinline__ void store(int64_t r, int64_t s, const C v[12]) const {
    S* p = data + r * 12 * V + s;
    if constexpr (FORM == CRK_FORM_FP16S) {
      float m = 0.f;
#pragma unroll
      for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].x), fabsf(v[c].y)));
      float inv = m > 0.f ? 1.0f / m : 0.f;
      scale[r * V + s] = m;
#pragma unroll
      for (int c = 0; c < 12; ++c) p[c * V] = __float22half2_rn(mk<float2>(v[c].x * inv, v[c].y * inv));
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) p[c * V] = v[c];
    }
  }
};

// Gauge links, [mu][9][V] (entry 3a+b of U_mu(x)); FP16S links are plain half2 (|U_ab| <= 1).
template <int FORM> struct GaugeView {
  using S = typename Prec<FORM>::store;
  using C = typename Prec<FORM>::cx;
  const S* data;
  int64_t V;
  __device__ __forceinline__ void load(int mu, int64_t s, C u[9]) const {
    const S* p = data + int64_t(mu) * 9 * V + s;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      if constexpr (FORM == CRK_FORM_FP16S) u[e] = __half22float2(p[e * V]);
      else u[e] = p[e * V];
    }
  }
};

}  // namespace crk
