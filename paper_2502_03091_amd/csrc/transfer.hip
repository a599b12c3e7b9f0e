// Restriction R = P^dag and prolongation P between level l and level l+1
// (paper, Sec. 2: R = P^dag; Sec. 3, Eq. (6): P is block diagonal, block j and
// chirality alpha holding the k left singular vectors u_i^(alpha) on Lambda_j).
//
//   (R v)(j)[alpha*k + i] = sum_{c', l} conj(P_{j,alpha}[i][c'*nb + l]) v(j*nb + l)[alpha*h + c']
//   (P w)(j*nb + l)[alpha*h + c'] = sum_i P_{j,alpha}[i][c'*nb + l] w(j)[alpha*k + i]
//
// One workgroup per (block, chirality).  Restriction stages row chunks of P
// and of the input in LDS and accumulates each output over the rows in order;
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

// Restriction as a blocked product out = P_{j,alpha}^dag v over row chunks of
// 64: the workgroup stages the chunk of P (k x 64) and of v (64 x 16 RHS) in
// LDS with coalesced loads (the next chunk's loads in flight while the current
// one is multiplied), then either thread (i-pair, rhs) accumulates its two
// outputs over the chunk (FMA form), or (MF, FP32) wavefront w multiplies rows
// 16w .. 16w+15 of the chunk on the matrix cores: two 16-row tiles of conj(P)
// times the 16-RHS tile, v_mfma_f32_16x16x4f32 with four real products per
// complex one, and the four wavefronts' tiles are added in LDS in wavefront
// order.  Either way every output has one fixed summation order.
constexpr int kRowChunk = 64;
constexpr int kRhsChunk = 16;
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <class T, bool MF>
__global__ __launch_bounds__(kT) void restrict_lds_kernel(TransferGeom g, const typename cplx_t<T>::type* __restrict__ P,
                                                          const typename cplx_t<T>::type* __restrict__ v,
                                                          typename cplx_t<T>::type* __restrict__ out, int nrhs) {
  using C = typename cplx_t<T>::type;
  static_assert(!MF || sizeof(T) == 4, "matrix-core restriction: FP32 only");
  __shared__ C Ps[32][kRowChunk + 1];
  __shared__ C Vs[kRowChunk][kRhsChunk];
  // partial tiles of wavefronts 1..3: [wave-1][row tile][re, im][accumulator entry][lane]
  __shared__ float red[MF ? kT / 64 - 1 : 1][2][2][4][MF ? 64 : 1];
  const int pair = blockIdx.x;
  const int64_t j = pair >> 1;
  const int alpha = pair & 1;
  const int nr = g.h * g.nb, k = g.k, N = 2 * k;
  const C* Pp = P + int64_t(pair) * k * nr;
  const int64_t jp = g.pos_c ? g.pos_c[j] : j;
  const int q = threadIdx.x % kRhsChunk, i0 = threadIdx.x / kRhsChunk, i1 = i0 + 16;
  // The chunk after the current one is loaded into registers while the current
  // one is multiplied (each thread stages the same entries of every chunk).
  constexpr int kPL = 32 * kRowChunk / kT, kVL2 = kRhsChunk * kRowChunk / kT;
  static_assert(32 * kRowChunk % kT == 0 && kRhsChunk * kRowChunk % kT == 0, "restriction staging");
  C pn[kPL], vn[kVL2];
  auto load_chunk = [&](int c0, int r0) {
#pragma unroll
    for (int u = 0; u < kPL; ++u) {
      const int e = int(threadIdx.x) + u * kT, i = e / kRowChunk, rr = e % kRowChunk;
      pn[u] = (i < k && c0 + rr < nr) ? Pp[int64_t(i) * nr + c0 + rr] : C{0, 0};
    }
#pragma unroll
    for (int u = 0; u < kVL2; ++u) {
      const int e = int(threadIdx.x) + u * kT, qq = e / kRowChunk, rr = e % kRowChunk, rho = c0 + rr;
      C val = C{0, 0};
      if (rho < nr && r0 + qq < nrhs) {
        const int cp = rho / g.nb, l = rho % g.nb;
        const int64_t site = j * g.nb + l;
        const int r = r0 + qq;
        val = v[g.aosoa ? aidx(r, alpha * g.h + cp, site, g.Vp, g.ncomp)
                        : int64_t(r) * g.vr + int64_t(alpha * g.h + cp) * g.vc + site * g.vs];
      }
      vn[u] = val;
    }
  };
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int r0 = 0; r0 < nrhs; r0 += kRhsChunk) {
    C a0 = C{0, 0}, a1 = C{0, 0};
    floatx4 are0[2], are1[2], aim0[2], aim1[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) are0[mt] = are1[mt] = aim0[mt] = aim1[mt] = floatx4{0, 0, 0, 0};
    load_chunk(0, r0);
    for (int c0 = 0; c0 < nr; c0 += kRowChunk) {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kPL; ++u) {
        const int e = int(threadIdx.x) + u * kT;
        Ps[e / kRowChunk][e % kRowChunk] = pn[u];
      }
#pragma unroll
      for (int u = 0; u < kVL2; ++u) {
        const int e = int(threadIdx.x) + u * kT;
        Vs[e % kRowChunk][e / kRowChunk] = vn[u];
      }
      __syncthreads();
      if (c0 + kRowChunk < nr) load_chunk(c0 + kRowChunk, r0);
      if constexpr (MF) {
        // lane (row = lane % 16, kq = lane / 16): A = conj(P)[row][k], B = v[k][rhs = lane % 16],
        // k = 16 wv + 4 ks + kq; conj(P) v = (Pr Vr + Pi Vi) + i (Pr Vi - Pi Vr)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int rr = 16 * wv + 4 * ks + (lane >> 4);
          const C b = Vs[rr][lane & 15];
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) {
            const C a = Ps[16 * mt + (lane & 15)][rr];
            are0[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, are0[mt], 0, 0, 0);
            aim0[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, aim0[mt], 0, 0, 0);
            are1[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, are1[mt], 0, 0, 0);
            aim1[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, b.x, aim1[mt], 0, 0, 0);
          }
        }
      } else {
#pragma unroll 8
        for (int rr = 0; rr < kRowChunk; ++rr) {
          const C x = Vs[rr][q];
          cfmac(a0, Ps[i0][rr], x);
          cfmac(a1, Ps[i1][rr], x);
        }
      }
    }
    if constexpr (MF) {
      if (wv > 0) {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            red[wv - 1][mt][0][e][lane] = are0[mt][e] + are1[mt][e];
            red[wv - 1][mt][1][e][lane] = aim0[mt][e] + aim1[mt][e];
          }
      }
      __syncthreads();
      if (wv == 0) {
        const int col = lane & 15;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            // accumulator entry e of lane: row 4 (lane / 16) + e of the tile, column lane % 16
            float re = are0[mt][e] + are1[mt][e], im = aim0[mt][e] + aim1[mt][e];
#pragma unroll
            for (int w = 0; w < kT / 64 - 1; ++w) {
              re += red[w][mt][0][e][lane];
              im += red[w][mt][1][e][lane];
            }
            const int i = 16 * mt + 4 * (lane >> 4) + e;
            if (i < k && r0 + col < nrhs) out[(jp * N + alpha * k + i) * nrhs + r0 + col] = C{re, im};
          }
      }
    } else if (r0 + q < nrhs) {
      if (i0 < k) out[(jp * N + alpha * k + i0) * nrhs + r0 + q] = a0;
      if (i1 < k) out[(jp * N + alpha * k + i1) * nrhs + r0 + q] = a1;
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
  if (prec == CRK_FORM_FP64)
    hipLaunchKernelGGL((restrict_lds_kernel<double, false>), grid, dim3(kT), 0, st, g, static_cast<const double2*>(P),
                       static_cast<const double2*>(fine), static_cast<double2*>(coarse), nrhs);
  else
    hipLaunchKernelGGL((restrict_lds_kernel<float, true>), grid, dim3(kT), 0, st, g, static_cast<const float2*>(P),
                       static_cast<const float2*>(fine), static_cast<float2*>(coarse), nrhs);
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
