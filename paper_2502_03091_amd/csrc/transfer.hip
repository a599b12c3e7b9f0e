// Restriction R = P^dag and prolongation P between level l and level l+1
// (paper, Sec. 2: R = P^dag; Sec. 3, Eq. (6): P is block diagonal, block j and
// chirality alpha holding the k left singular vectors u_i^(alpha) on Lambda_j).
//
//   (R v)(j)[alpha*k + i] = sum_{c', l} conj(P_{j,alpha}[i][c'*nb + l]) v(j*nb + l)[alpha*h + c']
//   (P w)(j*nb + l)[alpha*h + c'] = sum_i P_{j,alpha}[i][c'*nb + l] w(j)[alpha*k + i]
//
// One workgroup per (block, chirality).  Restriction splits the block's rows
// over 32 lanes and the k outputs over 8 lane groups, accumulating per-thread
// tiles in registers and summing the row slices with cross-lane shuffles;
// prolongation keeps the block's k x nrhs coarse values in LDS and lets each
// thread produce one fine row for up to 16 right-hand sides, so every entry of
// P is read from memory once per call (per 16 right-hand sides).  The fine side is addressed through
// (rhs, component, site) strides, covering both the rhs-outer fine layout
// and the rhs-inner coarse layout of an intermediate level.
#include "field.h"
#include "transfer.h"

namespace crk {

namespace {

constexpr int kT = 256;

// Restriction with register tiles: thread (i-group ig, row slice rs) accumulates
// TI x RC outputs over rows rs, rs+32, ...; the 32 row slices of an i-group are
// one half-wavefront and are summed with cross-lane shuffles.  P is read once,
// coalesced along the rows; each input entry is read by the 8 i-groups from cache.
template <class T, int TI, int RC>
__global__ __launch_bounds__(kT) void restrict_tiled_kernel(TransferGeom g,
                                                            const typename cplx_t<T>::type* __restrict__ P,
                                                            const typename cplx_t<T>::type* __restrict__ v,
                                                            typename cplx_t<T>::type* __restrict__ out, int nrhs) {
  using C = typename cplx_t<T>::type;
  const int pair = blockIdx.x;
  const int64_t j = pair >> 1;
  const int alpha = pair & 1;
  const int nr = g.h * g.nb, k = g.k, N = 2 * k;
  const int ig = threadIdx.x >> 5, rs = threadIdx.x & 31;
  const C* Pp = P + int64_t(pair) * k * nr;
  const int64_t jp = g.pos_c ? g.pos_c[j] : j;
  for (int r0 = 0; r0 < nrhs; r0 += RC) {
    C acc[TI][RC];
#pragma unroll
    for (int x = 0; x < TI; ++x)
#pragma unroll
      for (int q = 0; q < RC; ++q) acc[x][q] = C{0, 0};
    for (int rho = rs; rho < nr; rho += 32) {
      const int cp = rho / g.nb, l = rho % g.nb;
      const int64_t site = j * g.nb + l;
      C p[TI];
#pragma unroll
      for (int x = 0; x < TI; ++x) {
        const int i = ig * TI + x;
        p[x] = i < k ? Pp[int64_t(i) * nr + rho] : C{0, 0};
      }
#pragma unroll
      for (int q = 0; q < RC; ++q) {
        if (r0 + q < nrhs) {
          const int r = r0 + q;
          const C val = v[g.aosoa ? aidx(r, alpha * g.h + cp, site, g.Vp, g.ncomp)
                                  : int64_t(r) * g.vr + int64_t(alpha * g.h + cp) * g.vc + site * g.vs];
#pragma unroll
          for (int x = 0; x < TI; ++x) cfmac(acc[x][q], p[x], val);
        }
      }
    }
#pragma unroll
    for (int x = 0; x < TI; ++x)
#pragma unroll
      for (int q = 0; q < RC; ++q) {
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) {
          acc[x][q].x += __shfl_xor(acc[x][q].x, o);
          acc[x][q].y += __shfl_xor(acc[x][q].y, o);
        }
      }
    if (rs == 0) {
#pragma unroll
      for (int x = 0; x < TI; ++x) {
        const int i = ig * TI + x;
        if (i >= k) continue;
#pragma unroll
        for (int q = 0; q < RC; ++q)
          if (r0 + q < nrhs) out[(jp * N + alpha * k + i) * nrhs + r0 + q] = acc[x][q];
      }
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
    const int64_t site = j * g.nb + l;
    const int64_t base = g.aosoa ? aidx(0, alpha * g.h + cp, site, g.Vp, g.ncomp)
                                 : int64_t(alpha * g.h + cp) * g.vc + site * g.vs;
    const int64_t rstride = g.aosoa ? g.Vp * g.ncomp : g.vr;
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
          C* dst = v + base + int64_t(r0 + q) * rstride;
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
  CRK_REQUIRE(g.k >= 1 && g.k <= 32, "restriction: k must be in [1, 32]");
  const dim3 grid = dim3(unsigned(2 * g.nblocks));
  const int ti = (g.k + 7) / 8;
#define CRK_RESTRICT(T, TI, RC)                                                                               \
  hipLaunchKernelGGL((restrict_tiled_kernel<T, TI, RC>), grid, dim3(kT), 0, st, g,                            \
                     static_cast<const typename cplx_t<T>::type*>(P),                                         \
                     static_cast<const typename cplx_t<T>::type*>(fine),                                      \
                     static_cast<typename cplx_t<T>::type*>(coarse), nrhs)
  if (prec == CRK_FORM_FP64) {
    switch (ti) {
      case 1: CRK_RESTRICT(double, 1, 8); break;
      case 2: CRK_RESTRICT(double, 2, 8); break;
      case 3: CRK_RESTRICT(double, 3, 8); break;
      default: CRK_RESTRICT(double, 4, 8); break;
    }
  } else {
    switch (ti) {
      case 1: CRK_RESTRICT(float, 1, 16); break;
      case 2: CRK_RESTRICT(float, 2, 16); break;
      case 3: CRK_RESTRICT(float, 3, 16); break;
      default: CRK_RESTRICT(float, 4, 16); break;
    }
  }
#undef CRK_RESTRICT
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
