// Per-right-hand-side BLAS-1 kernels for fields of many RHS.
//
// A field set holds nrhs vectors of n complex entries each.  Two layouts are
// addressed through (rhs stride, element stride): fine fields are rhs-outer
// (element e of rhs r at r*n + e) and coarse fields rhs-inner (at e*nrhs + r).
// Reductions are deterministic: fixed per-thread element ranges, a fixed
// shuffle/LDS tree per workgroup, and a fixed-order final sum over workgroups.
#include "blas.h"
#include "field.h"

namespace crk {

namespace {

constexpr int kT = 256;

template <class T> struct C2;
template <> struct C2<double> { using t = double2; };
template <> struct C2<float> { using t = float2; };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Block-wide sum of NV doubles per thread into out[NV] (valid on thread 0).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh /* [NV][kT/64] */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double t = wave_sum(v[i]);
    if (lane == 0) sh[i * 4 + wid] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double t = 0;
      for (int w = 0; w < nw; ++w) t += sh[i * 4 + w];
      v[i] = t;
    }
  }
}

// partial[chunk][r][0..2] = (re, im) of sum conj(a) b, and sum |a|^2 over the chunk.
template <class T>
__global__ __launch_bounds__(kT) void dot_partial_kernel(const typename C2<T>::t* __restrict__ a,
                                                         const typename C2<T>::t* __restrict__ b, int64_t n, int nrhs,
                                                         int64_t rs, int64_t es, int64_t chunk,
                                                         double* __restrict__ partial) {
  __shared__ double sh[3 * 4];
  const int r = blockIdx.y;
  const int64_t e0 = int64_t(blockIdx.x) * chunk, e1 = min(n, e0 + chunk);
  double v[3] = {0, 0, 0};
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int64_t idx = int64_t(r) * rs + e * es;
    const auto x = a[idx];
    const auto y = b ? b[idx] : x;
    v[0] += double(x.x) * y.x + double(x.y) * y.y;
    v[1] += double(x.x) * y.y - double(x.y) * y.x;
    v[2] += double(x.x) * x.x + double(x.y) * x.y;
  }
  block_sum<3>(v, sh);
  if (threadIdx.x == 0) {
    double* p = partial + (int64_t(blockIdx.x) * nrhs + r) * 3;
    p[0] = v[0]; p[1] = v[1]; p[2] = v[2];
  }
}

// dot_partial_kernel for rhs-inner fields (entry e of rhs r at e*nrhs + r):
// workgroup per (chunk of kInnerChunk entries, group of up to 16 RHS), thread
// (l, r) with r fastest, so a wavefront reads contiguous RHS runs; thread (l, r)
// adds entries l, l + 64, ... of the chunk, the 64 lane sums of an RHS are
// added in lane order (independent of how many RHS share the field).
constexpr int kDotRhs = 16;

template <class T>
__global__ __launch_bounds__(64 * kDotRhs) void dot_partial_rg_kernel(const typename C2<T>::t* __restrict__ a,
                                                                      const typename C2<T>::t* __restrict__ b,
                                                                      int64_t n, int nrhs,
                                                                      double* __restrict__ partial) {
  __shared__ double sh[64][kDotRhs][3];  // [lane][rhs]: the RHS of a lane in different banks
  const int rg = min(kDotRhs, nrhs - int(blockIdx.y) * kDotRhs);
  const int t = threadIdx.x;
  const int rl = t % rg, l = t / rg;
  const int r = int(blockIdx.y) * kDotRhs + rl;
  if (l < 64) {
    double v0 = 0, v1 = 0, v2 = 0;
    for (int i = 0; i < kInnerChunk / 64; ++i) {
      const int64_t e = int64_t(blockIdx.x) * kInnerChunk + l + 64 * i;
      if (e >= n) break;
      const int64_t idx = e * nrhs + r;
      const auto x = a[idx];
      const auto y = b ? b[idx] : x;
      v0 += double(x.x) * y.x + double(x.y) * y.y;
      v1 += double(x.x) * y.y - double(x.y) * y.x;
      v2 += double(x.x) * x.x + double(x.y) * x.y;
    }
    sh[l][rl][0] = v0;
    sh[l][rl][1] = v1;
    sh[l][rl][2] = v2;
  }
  __syncthreads();
  if (t < 3 * rg) {
    const int rr = t / 3, v = t % 3;
    double s = 0;
    for (int k = 0; k < 64; ++k) s += sh[k][rr][v];
    partial[(int64_t(blockIdx.x) * nrhs + int(blockIdx.y) * kDotRhs + rr) * 3 + v] = s;
  }
}

// Chunk partials of (<a, b>, ||a||^2) for any layout (rhs-inner: the grouped kernel).
template <class T>
void launch_dot_partial(const void* a, const void* b, int64_t n, int nrhs, int64_t rs, int64_t es, int64_t chunk,
                        int64_t nch, double* partial, hipStream_t st) {
  using CT = typename C2<T>::t;
  if (es != 1 && rs == 1 && es == nrhs && chunk == kInnerChunk) {
    const dim3 g = dim3(unsigned(nch), unsigned((nrhs + kDotRhs - 1) / kDotRhs));
    hipLaunchKernelGGL(dot_partial_rg_kernel<T>, g, dim3(unsigned(64 * (nrhs < kDotRhs ? nrhs : kDotRhs))), 0, st,
                       static_cast<const CT*>(a), static_cast<const CT*>(b), n, nrhs, partial);
  } else {
    const dim3 g = dim3(unsigned(nch), unsigned(nrhs));
    hipLaunchKernelGGL(dot_partial_kernel<T>, g, dim3(kT), 0, st, static_cast<const CT*>(a),
                       static_cast<const CT*>(b), n, nrhs, rs, es, chunk, partial);
  }
  CRK_LAUNCH_CHECK();
}

// Sum partial[nchunk][nrhs][nv] over chunks in a fixed order; out[r][nv].
__global__ __launch_bounds__(kT) void reduce_partial_kernel(const double* __restrict__ partial, int64_t nchunk,
                                                            int nrhs, int nv, double* __restrict__ out) {
  __shared__ double sh[4];
  const int r = blockIdx.x / nv, c = blockIdx.x % nv;
  double v[1] = {0};
  // chunks i = t, t + T, t + 2T, ... added in that order, their loads issued 16 at a time
  constexpr int kU = 16;
  const int64_t T = blockDim.x;
  for (int64_t i0 = threadIdx.x; i0 < nchunk; i0 += kU * T) {
    double x[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = i0 + u * T;
      x[u] = i < nchunk ? partial[(i * nrhs + r) * nv + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (i0 + u * T < nchunk) v[0] += x[u];
  }
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) out[r * nv + c] = v[0];
}

__global__ void mr_alpha_kernel(const double* __restrict__ sums, int nrhs, double2* __restrict__ alpha) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const double qq = sums[3 * r + 2];
  alpha[r] = qq > 0 ? make_double2(sums[3 * r] / qq, sums[3 * r + 1] / qq) : make_double2(0, 0);
}

// r - a q for FP32 fields with each product and the difference rounded as
// written (the barrier keeps a q out of any fusion with the subtraction), so
// the one-sweep update and the deferred updates form the same residuals.
__device__ __forceinline__ float2 mr_next_f(float2 r, float2 a, float2 q) {
  float qx = fmaf(a.x, q.x, -(a.y * q.y)), qy = fmaf(a.y, q.x, a.x * q.y);
  asm volatile("" : "+v"(qx), "+v"(qy));
  return mk<float2>(r.x - qx, r.y - qy);
}
__device__ __forceinline__ double2 mr_next(double2 r, double2 a, double2 q) {
  double2 nr = r;
  const double2 qa = cmul(a, q);
  nr.x -= qa.x;
  nr.y -= qa.y;
  return nr;
}
__device__ __forceinline__ float2 mr_next(float2 r, float2 a, float2 q) { return mr_next_f(r, a, q); }

// r - a q for one component of an FP16-storage residual, each product and the
// difference rounded as written: the decoded r (a product with its site scale)
// is kept out of any fused multiply-add, so every kernel that forms the next
// residual gets the same bits whether or not it also uses r for psi.
__device__ __forceinline__ float2 mr_next_h(float2 r, float2 a, float2 q) {
  asm volatile("" : "+v"(r.x), "+v"(r.y));
  const float qx = fmaf(a.x, q.x, -(a.y * q.y)), qy = fmaf(a.x, q.y, a.y * q.x);
  return mk<float2>(r.x - qx, r.y - qy);
}

// psi += alpha r ;  r -= alpha q  with psi FP32 and r, q in FP16 storage: one
// thread per (site, rhs) of the fine AoSoA layout, the same complex arithmetic
// as mr_update_kernel<float>, the new r stored with its site's new scale.
__global__ __launch_bounds__(kT) void mr_update_h_kernel(float2* __restrict__ psi, FineView<CRK_FORM_FP16S> r,
                                                         FineView<CRK_FORM_FP16S> q,
                                                         const double2* __restrict__ alpha, int64_t V, int nrhs,
                                                         int upd_r) {
  const int64_t Vp = pad_sites(V);
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= Vp * nrhs) return;
  const int64_t rr = i / Vp, s = i % Vp;
  if (s >= V) return;  // padding sites are never read
  const double2 ad = alpha[rr];
  const float2 a = make_float2(float(ad.x), float(ad.y));
  float2 rv[12], qv[12];
  r.load(rr, s, rv);
  float2* pp = psi + aidx(rr, 0, s, Vp, 12);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    float2 p = pp[c * kVL];
    cfma(p, a, rv[c]);
    pp[c * kVL] = p;
  }
  if (!upd_r) return;
  q.load(rr, s, qv);
#pragma unroll
  for (int c = 0; c < 12; ++c) rv[c] = mr_next_h(rv[c], a, qv[c]);
  r.store(rr, s, rv);
}

// mr_update_ring_kernel<float> for rhs-outer fields with an even number of
// entries per RHS: two complex entries per thread, 16-byte accesses.
__global__ __launch_bounds__(kT) void mr_update_ring2_kernel(float4* __restrict__ psi, MrPending pend,
                                                             const float4* __restrict__ q,
                                                             float4* __restrict__ rnext, int64_t n2, int nrhs) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n2 * nrhs) return;
  const int rr = int(i / n2);
  const int last = pend.n - 1;
  float4 x[kMrMaxDefer];
#pragma unroll
  for (int j = 0; j < kMrMaxDefer; ++j)
    if (j <= last && (psi != nullptr || j == last)) x[j] = static_cast<const float4*>(pend.r[j])[i];
  if (rnext != nullptr) {
    float4 rk = x[0];
#pragma unroll
    for (int j = 1; j < kMrMaxDefer; ++j)
      if (j == last) rk = x[j];
    const double2 ad = pend.alpha[last][rr];
    const float2 a = make_float2(float(ad.x), float(ad.y));
    const float4 qv = q[i];
    const float2 n0 = mr_next_f(make_float2(rk.x, rk.y), a, make_float2(qv.x, qv.y));
    const float2 n1 = mr_next_f(make_float2(rk.z, rk.w), a, make_float2(qv.z, qv.w));
    rnext[i] = make_float4(n0.x, n0.y, n1.x, n1.y);
  }
  if (psi != nullptr) {
    const float4 pv = psi[i];
    float2 p0 = make_float2(pv.x, pv.y), p1 = make_float2(pv.z, pv.w);
#pragma unroll
    for (int j = 0; j < kMrMaxDefer; ++j) {
      if (j > last) break;
      const double2 ad = pend.alpha[j][rr];
      const float2 a = make_float2(float(ad.x), float(ad.y));
      cfma(p0, a, make_float2(x[j].x, x[j].y));
      cfma(p1, a, make_float2(x[j].z, x[j].w));
    }
    psi[i] = make_float4(p0.x, p0.y, p1.x, p1.y);
  }
}

// Deferred updates with psi FP32 and r, q in FP16 storage (one thread per
// site and RHS): rnext = r_k - alpha_k q stored with its new site scale, and
// psi += alpha_j r_j over the pending sweeps, the arithmetic of
// mr_update_h_kernel in the same order.
struct MrPendingH {
  FineView<CRK_FORM_FP16S> r[kMrMaxDefer];
  const double2* alpha[kMrMaxDefer];
  int n;
};
__global__ __launch_bounds__(kT) void mr_update_h_ring_kernel(float2* __restrict__ psi, MrPendingH pend,
                                                              FineView<CRK_FORM_FP16S> q,
                                                              FineView<CRK_FORM_FP16S> rnext, int64_t V, int nrhs) {
  const int64_t Vp = pad_sites(V);
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= Vp * nrhs) return;
  const int64_t rr = i / Vp, s = i % Vp;
  if (s >= V) return;  // padding sites are never read
  const int last = pend.n - 1;
  if (rnext.data != nullptr) {
    FineView<CRK_FORM_FP16S> rk = pend.r[0];
    const double2* ak = pend.alpha[0];
#pragma unroll
    for (int j = 1; j < kMrMaxDefer; ++j)
      if (j == last) {
        rk = pend.r[j];
        ak = pend.alpha[j];
      }
    const double2 ad = ak[rr];
    const float2 a = make_float2(float(ad.x), float(ad.y));
    float2 rv[12], qv[12];
    rk.load(rr, s, rv);
    q.load(rr, s, qv);
#pragma unroll
    for (int c = 0; c < 12; ++c) rv[c] = mr_next_h(rv[c], a, qv[c]);
    rnext.store(rr, s, rv);
  }
  if (psi == nullptr) return;
  float2* pp = psi + aidx(rr, 0, s, Vp, 12);
  float2 p[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) p[c] = pp[c * kVL];
#pragma unroll
  for (int j = 0; j < kMrMaxDefer; ++j) {
    if (j > last) break;
    const double2 ad = pend.alpha[j][rr];
    const float2 a = make_float2(float(ad.x), float(ad.y));
    float2 x[12];
    pend.r[j].load(rr, s, x);
#pragma unroll
    for (int c = 0; c < 12; ++c) cfma(p[c], a, x[c]);
  }
#pragma unroll
  for (int c = 0; c < 12; ++c) pp[c * kVL] = p[c];
}

// psi += alpha r ;  r -= alpha q    (rhs-outer layout, n entries per rhs)
template <class T>
__global__ __launch_bounds__(kT) void mr_update_kernel(typename C2<T>::t* __restrict__ psi,
                                                       typename C2<T>::t* __restrict__ r,
                                                       const typename C2<T>::t* __restrict__ q,
                                                       const double2* __restrict__ alpha, int64_t n, int nrhs,
                                                       int rhs_inner, int upd_r) {
  using CT = typename C2<T>::t;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  const int rr = rhs_inner ? int(i % nrhs) : int(i / n);
  const double2 ad = alpha[rr];
  const CT a = mk<CT>(T(ad.x), T(ad.y));
  const CT rv = r[i];
  CT p = psi[i];
  cfma(p, a, rv);
  psi[i] = p;
  if (!upd_r) return;
  r[i] = mr_next(rv, a, q[i]);
}

// rnext = r_k - alpha_k q; psi += alpha_j r_j over the pending sweeps (the
// per-sweep arithmetic of mr_update_kernel, in the same order).
template <class T>
__global__ __launch_bounds__(kT) void mr_update_ring_kernel(typename C2<T>::t* __restrict__ psi, MrPending pend,
                                                            const typename C2<T>::t* __restrict__ q,
                                                            typename C2<T>::t* __restrict__ rnext, int64_t n,
                                                            int nrhs, int rhs_inner) {
  using CT = typename C2<T>::t;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  const int rr = rhs_inner ? int(i % nrhs) : int(i / n);
  const int last = pend.n - 1;
  CT x[kMrMaxDefer];
#pragma unroll
  for (int j = 0; j < kMrMaxDefer; ++j)
    if (j <= last && (psi != nullptr || j == last)) x[j] = static_cast<const CT*>(pend.r[j])[i];
  if (rnext != nullptr) {
    CT rk = x[0];
#pragma unroll
    for (int j = 1; j < kMrMaxDefer; ++j)
      if (j == last) rk = x[j];
    const double2 ad = pend.alpha[last][rr];
    const CT a = mk<CT>(T(ad.x), T(ad.y));
    rnext[i] = mr_next(rk, a, q[i]);
  }
  if (psi != nullptr) {
    CT p = psi[i];
#pragma unroll
    for (int j = 0; j < kMrMaxDefer; ++j) {
      if (j > last) break;
      const double2 ad = pend.alpha[j][rr];
      const CT a = mk<CT>(T(ad.x), T(ad.y));
      cfma(p, a, x[j]);
    }
    psi[i] = p;
  }
}

// v[e * nrhs + r] *= f[r] (rhs-inner field of n entries per rhs); the product in FP64.
template <class T>
__global__ __launch_bounds__(kT) void scale_rhs_inner_kernel(typename C2<T>::t* __restrict__ v,
                                                             const double* __restrict__ f, int64_t n, int nrhs) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  const double a = f[i % nrhs];
  typename C2<T>::t x = v[i];
  x.x = T(double(x.x) * a);
  x.y = T(double(x.y) * a);
  v[i] = x;
}

__global__ void inv_sqrt_kernel(const double* __restrict__ sums, int nv, int comp, int n, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = sums[i * nv + comp];
  out[i] = s > 0 ? 1.0 / sqrt(s) : 0.0;
}

// ---------------------------------------------------------------- Philox4x32-10
// Counter-based generator of Salmon, Moraes, Dror, Shaw (SC'11): ten rounds of
// two 32x32->64 multiplies with the published multipliers and Weyl key bumps.
__device__ __forceinline__ void philox_round(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
  const uint64_t p0 = uint64_t(0xD2511F53u) * c[0];
  const uint64_t p1 = uint64_t(0xCD9E8D57u) * c[2];
  const uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
  const uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
  c[0] = hi1 ^ c[1] ^ k0;
  c[1] = lo1;
  c[2] = hi0 ^ c[3] ^ k1;
  c[3] = lo0;
}

__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    philox_round(c, k0, k1);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// One complex Gaussian (Re, Im ~ N(0,1)) per entry via Box-Muller on two
// 64-bit uniforms in (0, 1).
template <class T>
__global__ __launch_bounds__(kT) void gaussian_kernel(typename C2<T>::t* __restrict__ out, int64_t total,
                                                      uint64_t seed, uint32_t stream) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  uint32_t c[4] = {uint32_t(i), uint32_t(uint64_t(i) >> 32), stream, 0x5eedu};
  philox4x32_10(c, uint32_t(seed), uint32_t(seed >> 32));
  const double u1 = (double((uint64_t(c[0]) << 32 | c[1]) >> 11) + 0.5) * 0x1.0p-53;
  const double u2 = (double((uint64_t(c[2]) << 32 | c[3]) >> 11) + 0.5) * 0x1.0p-53;
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);
  out[i] = mk<typename C2<T>::t>(T(rad * cs), T(rad * sn));
}

int64_t chunk_for(int64_t n) {
  // enough workgroups to fill the chip, fixed by n only (deterministic)
  int64_t c = (n + 1023) / 1024;
  if (c < 4096) c = 4096;
  return c;
}

}  // namespace

int64_t rhs_dot_partials(int64_t n, bool inner) {
  const int64_t c = inner ? int64_t(kInnerChunk) : chunk_for(n);
  return (n + c - 1) / c;
}

int64_t rhs_dot_launch(int prec, const void* a, const void* b, int64_t n, int nrhs, int64_t rs, int64_t es,
                       double* partial, hipStream_t st) {
  const int64_t chunk = es != 1 ? int64_t(kInnerChunk) : chunk_for(n);
  const int64_t nch = (n + chunk - 1) / chunk;
  if (nrhs <= 0 || n <= 0) return nch;
  if (prec == CRK_FORM_FP64) launch_dot_partial<double>(a, b, n, nrhs, rs, es, chunk, nch, partial, st);
  else launch_dot_partial<float>(a, b, n, nrhs, rs, es, chunk, nch, partial, st);
  return nch;
}

void rhs_dot(int prec, const void* a, const void* b, int64_t n, int nrhs, int64_t rs, int64_t es, double* partial,
             double* out3, hipStream_t st) {
  if (nrhs <= 0 || n <= 0) return;
  // rhs-inner (coarse) fields: one element per thread, many small workgroups
  const int64_t chunk = es != 1 ? int64_t(kInnerChunk) : chunk_for(n);
  const int64_t nch = (n + chunk - 1) / chunk;
  if (prec == CRK_FORM_FP64) launch_dot_partial<double>(a, b, n, nrhs, rs, es, chunk, nch, partial, st);
  else launch_dot_partial<float>(a, b, n, nrhs, rs, es, chunk, nch, partial, st);
  reduce_partials(partial, nch, nrhs, 3, out3, st);
}

void reduce_partials(const double* partial, int64_t nchunk, int nrhs, int nv, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_partial_kernel, dim3(unsigned(nrhs * nv)), dim3(kT), 0, st, partial, nchunk, nrhs, nv, out);
  CRK_LAUNCH_CHECK();
}

void mr_alpha(const double* sums3, int nrhs, double2* alpha, hipStream_t st) {
  hipLaunchKernelGGL(mr_alpha_kernel, dim3(ceil_div(nrhs, 64)), dim3(64), 0, st, sums3, nrhs, alpha);
  CRK_LAUNCH_CHECK();
}

void mr_update(int prec, void* psi, void* r, const void* q, const double2* alpha, int64_t n, int nrhs, bool rhs_inner,
               hipStream_t st, bool update_r) {
  const dim3 g(ceil_div(n * nrhs, kT));
  if (prec == CRK_FORM_FP64)
    hipLaunchKernelGGL(mr_update_kernel<double>, g, dim3(kT), 0, st, static_cast<double2*>(psi),
                       static_cast<double2*>(r), static_cast<const double2*>(q), alpha, n, nrhs, int(rhs_inner),
                       int(update_r));
  else
    hipLaunchKernelGGL(mr_update_kernel<float>, g, dim3(kT), 0, st, static_cast<float2*>(psi),
                       static_cast<float2*>(r), static_cast<const float2*>(q), alpha, n, nrhs, int(rhs_inner),
                       int(update_r));
  CRK_LAUNCH_CHECK();
}

void mr_update_ring(int prec, void* psi, const MrPending& pend, const void* q, void* rnext, int64_t n, int nrhs,
                    bool rhs_inner, hipStream_t st) {
  CRK_REQUIRE(pend.n >= 1 && pend.n <= kMrMaxDefer, "mr_update_ring: 1 to 8 pending sweeps");
  if (n <= 0 || nrhs <= 0) return;
  bool pairs = prec != CRK_FORM_FP64 && !rhs_inner && n % 2 == 0;
  auto al16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  for (int j = 0; j < pend.n; ++j) pairs = pairs && al16(pend.r[j]);
  pairs = pairs && al16(psi) && al16(q) && al16(rnext);
  if (pairs) {
    hipLaunchKernelGGL(mr_update_ring2_kernel, dim3(ceil_div(n / 2 * nrhs, kT)), dim3(kT), 0, st,
                       static_cast<float4*>(psi), pend, static_cast<const float4*>(q), static_cast<float4*>(rnext),
                       n / 2, nrhs);
    CRK_LAUNCH_CHECK();
    return;
  }
  const dim3 g(ceil_div(n * nrhs, kT));
  if (prec == CRK_FORM_FP64)
    hipLaunchKernelGGL(mr_update_ring_kernel<double>, g, dim3(kT), 0, st, static_cast<double2*>(psi), pend,
                       static_cast<const double2*>(q), static_cast<double2*>(rnext), n, nrhs, int(rhs_inner));
  else
    hipLaunchKernelGGL(mr_update_ring_kernel<float>, g, dim3(kT), 0, st, static_cast<float2*>(psi), pend,
                       static_cast<const float2*>(q), static_cast<float2*>(rnext), n, nrhs, int(rhs_inner));
  CRK_LAUNCH_CHECK();
}

void MrSweeps::update(int prec, void* psi, const void* q, int it, int nsweeps, int64_t n, int nrhs, bool rhs_inner,
                      hipStream_t st) {
  const bool more = it + 1 < nsweeps;
  if (slots_.size() == 1) {
    mr_update(prec, psi, slots_[0], q, alpha(it), n, nrhs, rhs_inner, st, more);
    return;
  }
  ++pending_;
  const bool flush = pending_ == D_ || !more;
  MrPending pend{};
  pend.n = flush ? pending_ : 1;
  for (int j = 0; j < pend.n; ++j) {
    const int sw = it - pend.n + 1 + j;
    pend.r[j] = r(sw);
    pend.alpha[j] = alpha(sw);
  }
  mr_update_ring(prec, flush ? psi : nullptr, pend, q, more ? r(it + 1) : nullptr, n, nrhs, rhs_inner, st);
  if (flush) pending_ = 0;
}

void MrSweeps::update_fine_h(void* psi, const void* q, int it, int nsweeps, int64_t V, int nrhs, hipStream_t st) {
  const bool more = it + 1 < nsweeps;
  if (slots_.size() == 1) {
    mr_update_fine_h(psi, slots_[0], q, alpha(it), V, nrhs, st, more);
    return;
  }
  ++pending_;
  const bool flush = pending_ == D_ || !more;
  if (V > 0 && nrhs > 0) {
    MrPendingH pend{};
    pend.n = flush ? pending_ : 1;
    for (int j = 0; j < pend.n; ++j) {
      const int sw = it - pend.n + 1 + j;
      pend.r[j] = FineView<CRK_FORM_FP16S>(r(sw), V, nrhs);
      pend.alpha[j] = alpha(sw);
    }
    FineView<CRK_FORM_FP16S> qv(const_cast<void*>(q), V, nrhs), rn;
    if (more) rn = FineView<CRK_FORM_FP16S>(r(it + 1), V, nrhs);
    hipLaunchKernelGGL(mr_update_h_ring_kernel, dim3(ceil_div(pad_sites(V) * nrhs, kT)), dim3(kT), 0, st,
                       static_cast<float2*>(flush ? psi : nullptr), pend, qv, rn, V, nrhs);
    CRK_LAUNCH_CHECK();
  }
  if (flush) pending_ = 0;
}

void mr_update_fine_h(void* psi, void* r, const void* q, const double2* alpha, int64_t V, int nrhs, hipStream_t st,
                      bool update_r) {
  if (V <= 0 || nrhs <= 0) return;
  FineView<CRK_FORM_FP16S> rv(r, V, nrhs), qv(const_cast<void*>(q), V, nrhs);
  hipLaunchKernelGGL(mr_update_h_kernel, dim3(ceil_div(pad_sites(V) * nrhs, kT)), dim3(kT), 0, st,
                     static_cast<float2*>(psi), rv, qv, alpha, V, nrhs, int(update_r));
  CRK_LAUNCH_CHECK();
}

void scale_rhs_inner(int prec, void* v, const double* f, int64_t n, int nrhs, hipStream_t st) {
  if (n * nrhs <= 0) return;
  const dim3 g(unsigned(ceil_div(n * nrhs, int64_t(kT))));
  if (prec == CRK_FORM_FP64)
    hipLaunchKernelGGL(scale_rhs_inner_kernel<double>, g, dim3(kT), 0, st, static_cast<double2*>(v), f, n, nrhs);
  else
    hipLaunchKernelGGL(scale_rhs_inner_kernel<float>, g, dim3(kT), 0, st, static_cast<float2*>(v), f, n, nrhs);
  CRK_LAUNCH_CHECK();
}

void inv_sqrt(const double* sums, int nv, int comp, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(inv_sqrt_kernel, dim3(ceil_div(n, 64)), dim3(64), 0, st, sums, nv, comp, n, out);
  CRK_LAUNCH_CHECK();
}

void gaussian_fill(int prec, void* out, int64_t total, uint64_t seed, uint32_t stream, hipStream_t st) {
  if (total <= 0) return;
  const dim3 g(ceil_div(total, kT));
  if (prec == CRK_FORM_FP64)
    hipLaunchKernelGGL(gaussian_kernel<double>, g, dim3(kT), 0, st, static_cast<double2*>(out), total, seed, stream);
  else
    hipLaunchKernelGGL(gaussian_kernel<float>, g, dim3(kT), 0, st, static_cast<float2*>(out), total, seed, stream);
  CRK_LAUNCH_CHECK();
}

}  // namespace crk
