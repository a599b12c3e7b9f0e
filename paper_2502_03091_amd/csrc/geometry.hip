// Lattice geometry on the device: site order, neighbour tables, block maps,
// and the layout conversions between the host and the native device layouts.
//
// Lexicographic site index s = x0 + L0*(x1 + L1*(x2 + L2*x3)), periodic
// neighbours x +- mu.  With a blocking b (paper, Sec. 2: the domain
// decomposition Lambda_j whose blocks become coarse sites) the device order is
// block-major: position j*|b| + l with j the lexicographic index of floor(x/b)
// on the coarse lattice and l that of x mod b inside the block, so that every
// block-local operation (chiral split, SVD, P, Galerkin, transfers) reads one
// contiguous range of sites.
#include "field.h"
#include "kernels.h"

namespace crk {

namespace {

struct Dims { int L[4]; int b[4]; int use_block; };

__device__ __forceinline__ void coords_of(int64_t s, const int L[4], int c[4]) {
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) { c[mu] = int(s % L[mu]); s /= L[mu]; }
}
__device__ __forceinline__ int64_t lex_of(const int c[4], const int L[4]) {
  return c[0] + int64_t(L[0]) * (c[1] + int64_t(L[1]) * (c[2] + int64_t(L[2]) * c[3]));
}

__device__ __forceinline__ int64_t position(const int c[4], const Dims& d) {
  if (!d.use_block) return lex_of(c, d.L);
  int X[4], l[4], cd[4];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) { X[mu] = c[mu] / d.b[mu]; l[mu] = c[mu] % d.b[mu]; cd[mu] = d.L[mu] / d.b[mu]; }
  const int64_t nb = int64_t(d.b[0]) * d.b[1] * d.b[2] * d.b[3];
  return lex_of(X, cd) * nb + lex_of(l, d.b);
}

__global__ void geometry_kernel(Dims d, int64_t V, int* __restrict__ pos, int* __restrict__ inv, int* __restrict__ nbr) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= V) return;
  int c[4];
  coords_of(s, d.L, c);
  const int64_t p = position(c, d);
  pos[s] = int(p);
  inv[p] = int(s);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      int cc[4] = {c[0], c[1], c[2], c[3]};
      cc[mu] = (cc[mu] + (k == 0 ? 1 : d.L[mu] - 1)) % d.L[mu];
      nbr[int64_t(2 * mu + k) * V + p] = int(position(cc, d));
    }
  }
}

__global__ void block_map_kernel(Dims d, int64_t V, int* __restrict__ out) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= V) return;
  int c[4], X[4], l[4], cd[4];
  coords_of(s, d.L, c);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) { X[mu] = c[mu] / d.b[mu]; l[mu] = c[mu] % d.b[mu]; cd[mu] = d.L[mu] / d.b[mu]; }
  out[2 * s] = int(lex_of(X, cd));
  out[2 * s + 1] = int(lex_of(l, d.b));
}

template <int FORM>
__global__ void gauge_kernel(const double2* __restrict__ src, typename Prec<FORM>::store* __restrict__ dst,
                             const int* __restrict__ pos, int64_t V) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;  // over V*36
  if (i >= V * 36) return;
  const int64_t s = i / 36;
  const int me = int(i % 36), mu = me / 9, e = me % 9;
  const double2 u = src[i];
  const int64_t p = pos ? pos[s] : s;
  typename Prec<FORM>::store v;
  if constexpr (FORM == CRK_FORM_FP16S) v = __float22half2_rn(make_float2(float(u.x), float(u.y)));
  else v = ccast<typename Prec<FORM>::store>(u);
  dst[aidx(mu, e, p, pad_sites(V), 9)] = v;
}

// One thread per (rhs, site): gathers the ncomp components of one site.
template <int FORM>
__global__ void import_kernel(const double2* __restrict__ src, void* dst, const int* __restrict__ pos, int64_t V,
                              int ncomp, int nrhs) {
  using S = typename Prec<FORM>::store;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= V * nrhs) return;
  const int64_t r = i / V, s = i % V;
  const int64_t p = pos ? pos[s] : s;
  const int64_t Vp = pad_sites(V);
  const double2* in = src + (r * V + s) * ncomp;
  S* out = static_cast<S*>(dst) + aidx(r, 0, p, Vp, ncomp);
  if constexpr (FORM == CRK_FORM_FP16S) {
    float m = 0.f;
    for (int c = 0; c < ncomp; ++c) m = fmaxf(m, fmaxf(fabsf(float(in[c].x)), fabsf(float(in[c].y))));
    const float inv = m > 0.f ? 1.f / m : 0.f;
    float* sc = reinterpret_cast<float*>(static_cast<S*>(dst) + int64_t(nrhs) * ncomp * Vp);
    sc[r * Vp + p] = m;
    for (int c = 0; c < ncomp; ++c)
      out[c * kVL] = __float22half2_rn(make_float2(float(in[c].x) * inv, float(in[c].y) * inv));
  } else {
    for (int c = 0; c < ncomp; ++c) out[c * kVL] = ccast<S>(in[c]);
  }
}

template <int FORM>
__global__ void export_kernel(const void* src, double2* __restrict__ dst, const int* __restrict__ pos, int64_t V,
                              int ncomp, int nrhs) {
  using S = typename Prec<FORM>::store;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= V * nrhs) return;
  const int64_t r = i / V, s = i % V;
  const int64_t p = pos ? pos[s] : s;
  const int64_t Vp = pad_sites(V);
  const S* in = static_cast<const S*>(src) + aidx(r, 0, p, Vp, ncomp);
  double2* out = dst + (r * V + s) * ncomp;
  if constexpr (FORM == CRK_FORM_FP16S) {
    const float* sc = reinterpret_cast<const float*>(static_cast<const S*>(src) + int64_t(nrhs) * ncomp * Vp);
    const float m = sc[r * Vp + p];
    for (int c = 0; c < ncomp; ++c) {
      float2 f = __half22float2(in[c * kVL]);
      out[c] = make_double2(double(f.x * m), double(f.y * m));
    }
  } else {
    for (int c = 0; c < ncomp; ++c) out[c] = ccast<double2>(in[c * kVL]);
  }
}

template <int SF, int DF>
__global__ void convert_kernel(const void* src, void* dst, int64_t V, int ncomp, int nrhs) {
  using SS = typename Prec<SF>::store;
  using DS = typename Prec<DF>::store;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t Vp = pad_sites(V);
  if (i >= Vp * nrhs) return;
  const int64_t r = i / Vp, s = i % Vp;
  if (s >= V) return;  // padding sites are never read
  const SS* in = static_cast<const SS*>(src) + aidx(r, 0, s, Vp, ncomp);
  DS* out = static_cast<DS*>(dst) + aidx(r, 0, s, Vp, ncomp);
  const int64_t V_ = Vp;  // scales are [nrhs][Vp]
  float m = 1.f, inv = 1.f;
  if constexpr (SF == CRK_FORM_FP16S) {
    m = reinterpret_cast<const float*>(static_cast<const SS*>(src) + int64_t(nrhs) * ncomp * Vp)[r * V_ + s];
  }
  if constexpr (DF == CRK_FORM_FP16S) {
    float mx = 0.f;
    for (int c = 0; c < ncomp; ++c) {
      float2 f;
      if constexpr (SF == CRK_FORM_FP16S) { f = __half22float2(in[c * kVL]); f.x *= m; f.y *= m; }
      else f = ccast<float2>(in[c * kVL]);
      mx = fmaxf(mx, fmaxf(fabsf(f.x), fabsf(f.y)));
    }
    inv = mx > 0.f ? 1.f / mx : 0.f;
    reinterpret_cast<float*>(static_cast<DS*>(dst) + int64_t(nrhs) * ncomp * Vp)[r * V_ + s] = mx;
  }
  for (int c = 0; c < ncomp; ++c) {
    if constexpr (SF == CRK_FORM_FP16S) {
      float2 f = __half22float2(in[c * kVL]);
      f.x *= m; f.y *= m;
      if constexpr (DF == CRK_FORM_FP16S) out[c * kVL] = __float22half2_rn(make_float2(f.x * inv, f.y * inv));
      else out[c * kVL] = ccast<DS>(f);
    } else {
      if constexpr (DF == CRK_FORM_FP16S) {
        float2 f = ccast<float2>(in[c * kVL]);
        out[c * kVL] = __float22half2_rn(make_float2(f.x * inv, f.y * inv));
      } else {
        out[c * kVL] = ccast<DS>(in[c * kVL]);
      }
    }
  }
}

Dims make_dims(const int dims[4], const int* block) {
  Dims d{};
  for (int mu = 0; mu < 4; ++mu) { d.L[mu] = dims[mu]; d.b[mu] = block ? block[mu] : 1; }
  d.use_block = block != nullptr;
  return d;
}

int64_t vol(const int dims[4]) { return int64_t(dims[0]) * dims[1] * dims[2] * dims[3]; }

}  // namespace

void build_geometry(const int dims[4], const int* block, int* pos, int* inv, int* nbr, hipStream_t st) {
  const int64_t V = vol(dims);
  hipLaunchKernelGGL(geometry_kernel, dim3(ceil_div(V, 256)), dim3(256), 0, st, make_dims(dims, block), V, pos, inv,
                     nbr);
  CRK_LAUNCH_CHECK();
}

void build_block_map(const int dims[4], const int block[4], int* out_jl, hipStream_t st) {
  const int64_t V = vol(dims);
  hipLaunchKernelGGL(block_map_kernel, dim3(ceil_div(V, 256)), dim3(256), 0, st, make_dims(dims, block), V, out_jl);
  CRK_LAUNCH_CHECK();
}

void gauge_convert(int form, const double2* src, void* dst, const int* pos, int64_t V, hipStream_t st) {
  const dim3 g(ceil_div(V * 36, 256));
  switch (form) {
    case CRK_FORM_FP64:
      hipLaunchKernelGGL(gauge_kernel<CRK_FORM_FP64>, g, dim3(256), 0, st, src, static_cast<double2*>(dst), pos, V);
      break;
    case CRK_FORM_FP32:
      hipLaunchKernelGGL(gauge_kernel<CRK_FORM_FP32>, g, dim3(256), 0, st, src, static_cast<float2*>(dst), pos, V);
      break;
    case CRK_FORM_FP16S:
      hipLaunchKernelGGL(gauge_kernel<CRK_FORM_FP16S>, g, dim3(256), 0, st, src, static_cast<__half2*>(dst), pos, V);
      break;
    default: fail(CRK_EINVAL, "unknown precision form");
  }
  CRK_LAUNCH_CHECK();
}

void field_import(int form, const double2* src, void* dst, const int* pos, int64_t V, int ncomp, int nrhs,
                  hipStream_t st) {
  const dim3 g(ceil_div(V * nrhs, 256));
  if (V * nrhs == 0) return;
  switch (form) {
    case CRK_FORM_FP64: hipLaunchKernelGGL(import_kernel<CRK_FORM_FP64>, g, dim3(256), 0, st, src, dst, pos, V, ncomp, nrhs); break;
    case CRK_FORM_FP32: hipLaunchKernelGGL(import_kernel<CRK_FORM_FP32>, g, dim3(256), 0, st, src, dst, pos, V, ncomp, nrhs); break;
    case CRK_FORM_FP16S: hipLaunchKernelGGL(import_kernel<CRK_FORM_FP16S>, g, dim3(256), 0, st, src, dst, pos, V, ncomp, nrhs); break;
    default: fail(CRK_EINVAL, "unknown precision form");
  }
  CRK_LAUNCH_CHECK();
}

void field_export(int form, const void* src, double2* dst, const int* pos, int64_t V, int ncomp, int nrhs,
                  hipStream_t st) {
  const dim3 g(ceil_div(V * nrhs, 256));
  if (V * nrhs == 0) return;
  switch (form) {
    case CRK_FORM_FP64: hipLaunchKernelGGL(export_kernel<CRK_FORM_FP64>, g, dim3(256), 0, st, src, dst, pos, V, ncomp, nrhs); break;
    case CRK_FORM_FP32: hipLaunchKernelGGL(export_kernel<CRK_FORM_FP32>, g, dim3(256), 0, st, src, dst, pos, V, ncomp, nrhs); break;
    case CRK_FORM_FP16S: hipLaunchKernelGGL(export_kernel<CRK_FORM_FP16S>, g, dim3(256), 0, st, src, dst, pos, V, ncomp, nrhs); break;
    default: fail(CRK_EINVAL, "unknown precision form");
  }
  CRK_LAUNCH_CHECK();
}

void field_convert(int sf, const void* src, int df, void* dst, int64_t V, int ncomp, int nrhs, hipStream_t st) {
  const dim3 g(ceil_div(pad_sites(V) * nrhs, 256));
  if (V * nrhs == 0) return;
#define CRK_CONV(A, B) \
  if (sf == A && df == B) { hipLaunchKernelGGL((convert_kernel<A, B>), g, dim3(256), 0, st, src, dst, V, ncomp, nrhs); CRK_LAUNCH_CHECK(); return; }
  CRK_CONV(CRK_FORM_FP64, CRK_FORM_FP32)
  CRK_CONV(CRK_FORM_FP64, CRK_FORM_FP16S)
  CRK_CONV(CRK_FORM_FP32, CRK_FORM_FP64)
  CRK_CONV(CRK_FORM_FP16S, CRK_FORM_FP64)
  CRK_CONV(CRK_FORM_FP32, CRK_FORM_FP16S)
  CRK_CONV(CRK_FORM_FP16S, CRK_FORM_FP32)
  CRK_CONV(CRK_FORM_FP64, CRK_FORM_FP64)
  CRK_CONV(CRK_FORM_FP32, CRK_FORM_FP32)
#undef CRK_CONV
  fail(CRK_EINVAL, "unsupported field conversion");
}

}  // namespace crk
