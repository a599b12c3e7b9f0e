// Clover (Sheikholeslami-Wohlert) site term of the Wilson-clover operator.
//
// The paper's ensembles use clover actions (Sec. 4) without writing the term
// out; the standard form is used, added to the Wilson site term:
//   X(x) = (m0 + sum_mu w_mu) 1 + C(x),
//   C(x) = -(c_sw/2) sum_{mu<nu} w_mu w_nu sigma_{mu nu} (x) F_{mu nu}(x),
//   F_{mu nu} = (1/8i) [(Q - Q^dag) - tr(Q - Q^dag)/3],
// Q_{mu nu}(x) the four counter-clockwise plaquettes of the (mu, nu) plane at x.
// In the chiral basis (gamma5 = diag(1, 1, -1, -1)) every sigma_{mu nu} = i
// gamma_mu gamma_nu (mu != nu) is block diagonal with Pauli-matrix blocks:
//   (x,y): -s3, -s3   (x,z): +s2, +s2   (y,z): -s1, -s1
//   (x,t): +s1, -s1   (y,t): +s2, -s2   (z,t): +s3, -s3
// (first block: spins 1,2 = chirality 0; second: spins 3,4 = chirality 1), so
// X(x) is two Hermitian 6 x 6 blocks X_alpha, row/column index 3*spin' + colour.
//
// Storage: entry e = 36*alpha + 6*r + c of site x.  clover_compute writes the
// FP64 blocks in lexicographic site order ([V][72] complex128); clover_convert
// lays them out like the spinors (site-vectorised, 72 "components", sites at
// their device positions) in the storage of a form (FP64 double2; FP32 and
// FP16S float2).
#include "clover.h"
#include "field.h"

namespace crk {

namespace {

struct Dims { int L[4]; };

__device__ __forceinline__ int64_t shift_site(int64_t s, int mu, int d, const Dims& D) {
  int c[4];
  int64_t r = s;
#pragma unroll
  for (int m = 0; m < 4; ++m) { c[m] = int(r % D.L[m]); r /= D.L[m]; }
  c[mu] = (c[mu] + d + D.L[mu]) % D.L[mu];
  return c[0] + int64_t(D.L[0]) * (c[1] + int64_t(D.L[1]) * (c[2] + int64_t(D.L[2]) * c[3]));
}

__device__ __forceinline__ void ld3(const double2* U, int64_t x, int mu, double2 (&m)[9]) {
  const double2* p = U + (x * 4 + mu) * 9;
#pragma unroll
  for (int e = 0; e < 9; ++e) m[e] = p[e];
}
__device__ __forceinline__ void dag3(const double2 (&a)[9], double2 (&b)[9]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) b[3 * i + j] = cconj(a[3 * j + i]);
}
__device__ __forceinline__ void mul3(const double2 (&a)[9], const double2 (&b)[9], double2 (&c)[9]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 t = make_double2(0, 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) cfma(t, a[3 * i + k], b[3 * k + j]);
      c[3 * i + j] = t;
    }
}
// acc += a b c d
__device__ __forceinline__ void add_leaf(const double2 (&a)[9], const double2 (&b)[9], const double2 (&c)[9],
                                         const double2 (&d)[9], double2 (&acc)[9]) {
  double2 t1[9], t2[9], t3[9];
  mul3(a, b, t1);
  mul3(t1, c, t2);
  mul3(t2, d, t3);
#pragma unroll
  for (int e = 0; e < 9; ++e) acc[e] = acc[e] + t3[e];
}

constexpr int kPlaneMu[6] = {0, 0, 1, 0, 1, 2};
constexpr int kPlaneNu[6] = {1, 2, 2, 3, 3, 3};

// F_{mu nu}(x) for one (site, plane), stored [V][6][9].
__global__ void field_strength_kernel(const double2* __restrict__ U, Dims D, int64_t V, double2* __restrict__ F) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= V * 6) return;
  const int64_t x = i / 6;
  const int p = int(i % 6);
  const int mu = kPlaneMu[p], nu = kPlaneNu[p];
  const int64_t xpm = shift_site(x, mu, +1, D), xpn = shift_site(x, nu, +1, D);
  const int64_t xmm = shift_site(x, mu, -1, D), xmn = shift_site(x, nu, -1, D);
  const int64_t xmm_pn = shift_site(xmm, nu, +1, D), xmm_mn = shift_site(xmm, nu, -1, D);
  const int64_t xmn_pm = shift_site(xmn, mu, +1, D);
  double2 a[9], b[9], c[9], d[9], q[9], t[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) q[e] = make_double2(0, 0);
  // x -> x+mu -> x+mu+nu -> x+nu -> x
  ld3(U, x, mu, a); ld3(U, xpm, nu, b); ld3(U, xpn, mu, t); dag3(t, c); ld3(U, x, nu, t); dag3(t, d);
  add_leaf(a, b, c, d, q);
  // x -> x+nu -> x+nu-mu -> x-mu -> x
  ld3(U, x, nu, a); ld3(U, xmm_pn, mu, t); dag3(t, b); ld3(U, xmm, nu, t); dag3(t, c); ld3(U, xmm, mu, d);
  add_leaf(a, b, c, d, q);
  // x -> x-mu -> x-mu-nu -> x-nu -> x
  ld3(U, xmm, mu, t); dag3(t, a); ld3(U, xmm_mn, nu, t); dag3(t, b); ld3(U, xmm_mn, mu, c); ld3(U, xmn, nu, d);
  add_leaf(a, b, c, d, q);
  // x -> x-nu -> x-nu+mu -> x+mu -> x
  ld3(U, xmn, nu, t); dag3(t, a); ld3(U, xmn, mu, b); ld3(U, xmn_pm, nu, c); ld3(U, x, mu, t); dag3(t, d);
  add_leaf(a, b, c, d, q);
  // A = Q - Q^dag, traceless part, F = A / (8i)
  double2 A[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int s = 0; s < 3; ++s) A[3 * r + s] = q[3 * r + s] - cconj(q[3 * s + r]);
  const double2 tr = make_double2((A[0].x + A[4].x + A[8].x) / 3.0, (A[0].y + A[4].y + A[8].y) / 3.0);
  A[0] = A[0] - tr;
  A[4] = A[4] - tr;
  A[8] = A[8] - tr;
  double2* out = F + (x * 6 + p) * 9;
#pragma unroll
  for (int e = 0; e < 9; ++e) out[e] = make_double2(A[e].y / 8.0, -A[e].x / 8.0);  // (x + iy) / (8i)
}

// Pauli block s_alpha(plane)[s][s'] of sigma_{mu nu} for chirality alpha.
__device__ __forceinline__ double2 sigma_block(int p, int alpha, int s, int t) {
  // plane p: 0 (x,y) -s3; 1 (x,z) +s2; 2 (y,z) -s1; 3 (x,t) +-s1; 4 (y,t) +-s2; 5 (z,t) +-s3
  const int pauli = p == 0 ? 3 : p == 1 ? 2 : p == 2 ? 1 : p - 2;
  double sign = p == 0 || p == 2 ? -1.0 : 1.0;
  if (p >= 3 && alpha == 1) sign = -sign;
  double2 v = make_double2(0, 0);
  if (pauli == 1) v = make_double2(s != t ? 1.0 : 0.0, 0.0);
  else if (pauli == 2) v = make_double2(0.0, s == t ? 0.0 : (s == 0 ? -1.0 : 1.0));
  else v = make_double2(s == t ? (s == 0 ? 1.0 : -1.0) : 0.0, 0.0);
  return cscale(v, sign);
}

// Row r of X_alpha(x) for one (site, alpha, r).
__global__ void clover_assemble_kernel(const double2* __restrict__ F, int64_t V, double c_sw, double4 w, double diag,
                                       double2* __restrict__ X) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= V * 12) return;
  const int64_t x = i / 12;
  const int alpha = int(i % 12) / 6, r = int(i % 6);
  const int s = r / 3, a = r % 3;
  const double wv[4] = {w.x, w.y, w.z, w.w};
  double2 row[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) row[c] = make_double2(c == r ? diag : 0.0, 0.0);
  for (int p = 0; p < 6; ++p) {
    const double coef = -0.5 * c_sw * wv[kPlaneMu[p]] * wv[kPlaneNu[p]];
    const double2* f = F + (x * 6 + p) * 9;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const double2 sg = cscale(sigma_block(p, alpha, s, t), coef);
#pragma unroll
      for (int b = 0; b < 3; ++b) cfma(row[3 * t + b], sg, f[3 * a + b]);
    }
  }
  double2* out = X + x * 72 + 36 * alpha + 6 * r;
#pragma unroll
  for (int c = 0; c < 6; ++c) out[c] = row[c];
}

template <class S>
__global__ void clover_convert_kernel(const double2* __restrict__ X, S* __restrict__ dst, const int* __restrict__ pos,
                                      int64_t V) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= V * 72) return;
  const int64_t x = i / 72;
  const int e = int(i % 72);
  const int64_t p = pos ? pos[x] : x;
  const double2 v = X[i];
  S o;
  o.x = decltype(o.x)(v.x);
  o.y = decltype(o.y)(v.y);
  dst[aidx(0, e, p, pad_sites(V), 72)] = o;
}

}  // namespace

size_t clover_bytes(int form, int64_t V) {
  return (form == CRK_FORM_FP64 ? sizeof(double2) : sizeof(float2)) * 72 * size_t(pad_sites(V));
}

void clover_compute(const double2* U, const int dims[4], double c_sw, const double w[4], double diag, double2* X,
                    hipStream_t st) {
  Dims D;
  for (int mu = 0; mu < 4; ++mu) D.L[mu] = dims[mu];
  const int64_t V = int64_t(dims[0]) * dims[1] * dims[2] * dims[3];
  DevBuf F(sizeof(double2) * 54 * size_t(V));
  hipLaunchKernelGGL(field_strength_kernel, dim3(ceil_div(V * 6, 256)), dim3(256), 0, st, U, D, V, F.as<double2>());
  CRK_LAUNCH_CHECK();
  hipLaunchKernelGGL(clover_assemble_kernel, dim3(ceil_div(V * 12, 256)), dim3(256), 0, st, F.as<double2>(), V, c_sw,
                     make_double4(w[0], w[1], w[2], w[3]), diag, X);
  CRK_LAUNCH_CHECK();
  CRK_HIP(hipStreamSynchronize(st));  // F is freed at scope exit
}

void clover_convert(int form, const double2* X, void* dst, const int* pos, int64_t V, hipStream_t st) {
  const dim3 g(ceil_div(V * 72, 256));
  if (form == CRK_FORM_FP64)
    hipLaunchKernelGGL(clover_convert_kernel<double2>, g, dim3(256), 0, st, X, static_cast<double2*>(dst), pos, V);
  else
    hipLaunchKernelGGL(clover_convert_kernel<float2>, g, dim3(256), 0, st, X, static_cast<float2*>(dst), pos, V);
  CRK_LAUNCH_CHECK();
}

}  // namespace crk
