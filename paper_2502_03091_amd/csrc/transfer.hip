// Restriction R = P^dag and prolongation P between level l and level l+1
// (paper, Sec. 2: R = P^dag; Sec. 3, Eq. (6): P is block diagonal, block j and
// chirality alpha holding the k left singular vectors u_i^(alpha) on Lambda_j).
//
//   (R v)(j)[alpha*k + i] = sum_{c', l} conj(P_{j,alpha}[i][c'*nb + l]) v(j*nb + l)[alpha*h + c']
//   (P w)(j*nb + l)[alpha*h + c'] = sum_i P_{j,alpha}[i][c'*nb + l] w(j)[alpha*k + i]
//
// One workgroup per (block, chirality).  Restriction stages a chunk of P and
// of the input rows in LDS and accumulates the k x nrhs outputs in registers;
// prolongation keeps the block's k x nrhs coarse values in LDS and lets each
// thread produce one fine row for up to 16 right-hand sides, so every entry of
// P is read from memory once per call.  The fine side is addressed through
// (rhs, component, site) strides, covering both the rhs-outer fine layout
// and the rhs-inner coarse layout of an intermediate level.
#include "transfer.h"

namespace crk {

namespace {

constexpr int kT = 256;
constexpr int kCh = 64;
constexpr int kMaxOut = 16;  // outputs per thread: k * nrhs <= 4096

template <class T>
__global__ __launch_bounds__(kT) void restrict_kernel(TransferGeom g, const typename cplx_t<T>::type* __restrict__ P,
                                                      const typename cplx_t<T>::type* __restrict__ v,
                                                      typename cplx_t<T>::type* __restrict__ out, int nrhs) {
  using C = typename cplx_t<T>::type;
  extern __shared__ unsigned char smem[];
  C* Ps = reinterpret_cast<C*>(smem);     // [k][kCh]
  C* Vs = Ps + g.k * kCh;                 // [nrhs][kCh]
  const int pair = blockIdx.x;
  const int64_t j = pair >> 1;
  const int alpha = pair & 1;
  const int nr = g.h * g.nb, k = g.k, nout = k * nrhs;
  const C* Pp = P + int64_t(pair) * k * nr;
  C acc[kMaxOut];
#pragma unroll
  for (int o = 0; o < kMaxOut; ++o) acc[o] = C{0, 0};
  for (int r0 = 0; r0 < nr; r0 += kCh) {
    const int nrows = min(kCh, nr - r0);
    __syncthreads();
    for (int e = threadIdx.x; e < k * kCh; e += blockDim.x) {
      const int i = e / kCh, c = e % kCh;
      Ps[e] = c < nrows ? Pp[int64_t(i) * nr + r0 + c] : C{0, 0};
    }
    for (int e = threadIdx.x; e < nrhs * kCh; e += blockDim.x) {
      int r, c;
      if (g.vr == 1) { r = e % nrhs; c = e / nrhs; } else { c = e % kCh; r = e / kCh; }
      C val{0, 0};
      if (c < nrows) {
        const int rho = r0 + c, cp = rho / g.nb, l = rho % g.nb;
        val = v[int64_t(r) * g.vr + int64_t(alpha * g.h + cp) * g.vc + (j * g.nb + l) * g.vs];
      }
      Vs[r * kCh + c] = val;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMaxOut; ++q) {
      const int o = threadIdx.x + q * kT;
      if (o < nout) {
        const int i = o / nrhs, r = o % nrhs;
        C a = acc[q];
        for (int c = 0; c < nrows; ++c) cfmac(a, Ps[i * kCh + c], Vs[r * kCh + c]);
        acc[q] = a;
      }
    }
  }
  const int64_t jp = g.pos_c ? g.pos_c[j] : j;
  const int N = 2 * k;
#pragma unroll
  for (int q = 0; q < kMaxOut; ++q) {
    const int o = threadIdx.x + q * kT;
    if (o < nout) {
      const int i = o / nrhs, r = o % nrhs;
      out[(jp * N + alpha * k + i) * nrhs + r] = acc[q];
    }
  }
}

template <class T>
__global__ __launch_bounds__(kT) void prolong_kernel(TransferGeom g, const typename cplx_t<T>::type* __restrict__ P,
                                                     const typename cplx_t<T>::type* __restrict__ w,
                                                     typename cplx_t<T>::type* __restrict__ v, int nrhs, int add) {
  using C = typename cplx_t<T>::type;
  extern __shared__ unsigned char smem[];
  C* Ws = reinterpret_cast<C*>(smem);  // [k][nrhs]
  const int pair = blockIdx.x;
  const int64_t j = pair >> 1;
  const int alpha = pair & 1;
  const int nr = g.h * g.nb, k = g.k, N = 2 * k;
  const int64_t jp = g.pos_c ? g.pos_c[j] : j;
  for (int e = threadIdx.x; e < k * nrhs; e += blockDim.x) {
    const int i = e / nrhs, r = e % nrhs;
    Ws[e] = w[(jp * N + alpha * k + i) * nrhs + r];
  }
  __syncthreads();
  const C* Pp = P + int64_t(pair) * k * nr;
  for (int rho = threadIdx.x; rho < nr; rho += blockDim.x) {
    const int cp = rho / g.nb, l = rho % g.nb;
    const int64_t base = int64_t(alpha * g.h + cp) * g.vc + (j * g.nb + l) * g.vs;
    for (int r0 = 0; r0 < nrhs; r0 += 16) {
      C acc[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = C{0, 0};
      for (int i = 0; i < k; ++i) {
        const C p = Pp[int64_t(i) * nr + rho];
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (r0 + q < nrhs) cfma(acc[q], p, Ws[i * nrhs + r0 + q]);
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        if (r0 + q < nrhs) {
          C* dst = v + base + int64_t(r0 + q) * g.vr;
          *dst = add ? (*dst + acc[q]) : acc[q];
        }
      }
    }
  }
}

// Dynamic LDS above 64 KiB must be enabled per kernel (gfx950: 160 KiB per workgroup,
// static LDS included).
template <class K> void allow_lds(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return;
  CRK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(bytes)));
}

}  // namespace

void transfer_restrict(int prec, const TransferGeom& g, const void* P, const void* fine, void* coarse, int nrhs,
                       hipStream_t st) {
  if (nrhs <= 0) return;
  CRK_REQUIRE(g.k * nrhs <= kMaxOut * kT, "restriction: k * nrhs above 4096");
  const dim3 grid = dim3(unsigned(2 * g.nblocks));
  if (prec == CRK_FORM_FP64) {
    const size_t lds = sizeof(double2) * size_t(g.k + nrhs) * kCh;
    allow_lds(restrict_kernel<double>, lds);
    hipLaunchKernelGGL(restrict_kernel<double>, grid, dim3(kT), lds, st, g, static_cast<const double2*>(P),
                       static_cast<const double2*>(fine), static_cast<double2*>(coarse), nrhs);
  } else {
    const size_t lds = sizeof(float2) * size_t(g.k + nrhs) * kCh;
    allow_lds(restrict_kernel<float>, lds);
    hipLaunchKernelGGL(restrict_kernel<float>, grid, dim3(kT), lds, st, g, static_cast<const float2*>(P),
                       static_cast<const float2*>(fine), static_cast<float2*>(coarse), nrhs);
  }
  CRK_LAUNCH_CHECK();
}

void transfer_prolong(int prec, const TransferGeom& g, const void* P, const void* coarse, void* fine, int nrhs,
                      bool add, hipStream_t st) {
  if (nrhs <= 0) return;
  const dim3 grid = dim3(unsigned(2 * g.nblocks));
  if (prec == CRK_FORM_FP64) {
    const size_t lds = sizeof(double2) * size_t(g.k) * nrhs;
    allow_lds(prolong_kernel<double>, lds);
    hipLaunchKernelGGL(prolong_kernel<double>, grid, dim3(kT), lds, st, g, static_cast<const double2*>(P),
                       static_cast<const double2*>(coarse), static_cast<double2*>(fine), nrhs, int(add));
  } else {
    const size_t lds = sizeof(float2) * size_t(g.k) * nrhs;
    allow_lds(prolong_kernel<float>, lds);
    hipLaunchKernelGGL(prolong_kernel<float>, grid, dim3(kT), lds, st, g, static_cast<const float2*>(P),
                       static_cast<const float2*>(coarse), static_cast<float2*>(fine), nrhs, int(add));
  }
  CRK_LAUNCH_CHECK();
}

}  // namespace crk
