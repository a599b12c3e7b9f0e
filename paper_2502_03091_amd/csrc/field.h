// Precision forms and native device field layouts.
//
// Fine-level fields are site-vectorised: sites are grouped in chunks of 64
// (one wavefront), and within a chunk each component is a contiguous run of
// 64 complex values.  Entry (r, c, s) of a field set with ncomp components
// lives at complex index  (r*Vp + 64*floor(s/64))*ncomp + 64*c + s%64  with
// Vp = V rounded up to 64.  A wavefront therefore reads one site's 12
// components as twelve 512-byte runs of one contiguous 6 KiB block (FP32),
// which keeps DRAM pages and address translations local.  Gauge links use the
// same layout with "rhs" = direction mu and 9 components (entry 3a+b).
// FP16S stores half2 values of x/scale with one fp32 scale per (r, s), the
// largest |re|, |im| of that site's 24 reals, scales laid out [r][Vp].
#pragma once

#include "common.h"

namespace crk {

template <int FORM> struct Prec;
template <> struct Prec<CRK_FORM_FP64> { using real = double; using cx = double2; using store = double2; };
template <> struct Prec<CRK_FORM_FP32> { using real = float; using cx = float2; using store = float2; };
template <> struct Prec<CRK_FORM_FP16S> { using real = float; using cx = float2; using store = __half2; };

constexpr int kVL = 64;  // sites per vector chunk

__host__ __device__ __forceinline__ int64_t pad_sites(int64_t V) { return (V + kVL - 1) / kVL * kVL; }

// complex-entry index of component c of site s of set r (AoSoA, ncomp components)
__host__ __device__ __forceinline__ int64_t aidx(int64_t r, int c, int64_t s, int64_t Vp, int ncomp) {
  return (r * Vp + (s & ~int64_t(kVL - 1))) * ncomp + int64_t(c) * kVL + (s & (kVL - 1));
}

inline size_t store_bytes(int form) { return form == CRK_FORM_FP64 ? 16 : form == CRK_FORM_FP32 ? 8 : 4; }

// Bytes of a fine field set: data plus (FP16S) scales, sites padded to 64.
inline size_t fine_field_bytes(int form, int64_t V, int64_t nrhs, int ncomp = 12) {
  const size_t Vp = size_t(pad_sites(V));
  size_t b = store_bytes(form) * size_t(nrhs) * size_t(ncomp) * Vp;
  if (form == CRK_FORM_FP16S) b += sizeof(float) * size_t(nrhs) * Vp;
  return b;
}

template <int FORM> struct FineView {
  using S = typename Prec<FORM>::store;
  using C = typename Prec<FORM>::cx;
  S* data;
  float* scale;  // FP16S only: [nrhs][Vp]
  int64_t Vp;

  __host__ __device__ FineView() : data(nullptr), scale(nullptr), Vp(0) {}
  __host__ FineView(void* base, int64_t V, int64_t nrhs)
      : data(static_cast<S*>(base)), scale(nullptr), Vp(pad_sites(V)) {
    if (FORM == CRK_FORM_FP16S)
      scale = reinterpret_cast<float*>(static_cast<char*>(base) + sizeof(S) * size_t(nrhs) * 12 * size_t(Vp));
  }

  __device__ __forceinline__ void load(int64_t r, int64_t s, C v[12]) const {
    const S* p = data + aidx(r, 0, s, Vp, 12);
    if constexpr (FORM == CRK_FORM_FP16S) {
      const float sc = scale[r * Vp + s];
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const float2 f = __half22float2(p[c * kVL]);
        v[c] = mk<float2>(f.x * sc, f.y * sc);
      }
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) v[c] = p[c * kVL];
    }
  }

  __device__ __forceinline__ void store(int64_t r, int64_t s, const C v[12]) const {
    S* p = data + aidx(r, 0, s, Vp, 12);
    if constexpr (FORM == CRK_FORM_FP16S) {
      float m = 0.f;
#pragma unroll
      for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].x), fabsf(v[c].y)));
      const float inv = m > 0.f ? 1.0f / m : 0.f;
      scale[r * Vp + s] = m;
#pragma unroll
      for (int c = 0; c < 12; ++c) p[c * kVL] = __float22half2_rn(mk<float2>(v[c].x * inv, v[c].y * inv));
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) p[c * kVL] = v[c];
    }
  }
};

// Gauge links U_mu(x)[a][b] at aidx(mu, 3a+b, x, Vp, 9); FP16S links are plain half2 (|U_ab| <= 1).
template <int FORM> struct GaugeView {
  using S = typename Prec<FORM>::store;
  using C = typename Prec<FORM>::cx;
  const S* data;
  int64_t Vp;
  __device__ __forceinline__ void load(int mu, int64_t s, C u[9]) const {
    const S* p = data + aidx(mu, 0, s, Vp, 9);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      if constexpr (FORM == CRK_FORM_FP16S) u[e] = __half22float2(p[e * kVL]);
      else u[e] = p[e * kVL];
    }
  }
};

inline size_t gauge_bytes(int form, int64_t V) { return store_bytes(form) * 36 * size_t(pad_sites(V)); }

}  // namespace crk
