// Coarse-level stencil operator on the matrix cores (paper, Sec. 2: the coarse
// operator D_{l+1} = R D_l P is a nearest-neighbour stencil with 2k components
// per coarse site; applying it over many right-hand sides is a batch of dense
// complex 2k x 2k by 2k x nrhs products).
//
//   (D_c v)(j) = X(j) v(j) + sum_mu [ Y_{+mu}(j) v(j+mu) + Y_{-mu}(j) v(j-mu) ]
//
// One wavefront computes a 16 x 16 output tile (16 rows of one coarse site, 16
// right-hand sides), looping over the nine links and over K in steps of 4
// with v_mfma_{f32,f64}_16x16x4: a complex product is four real MFMAs
// (re += Ar Br - Ai Bi, im += Ar Bi + Ai Br).  Links are column-major 2k x 2k
// blocks, so the 16 rows an A operand needs are one contiguous 16-entry run;
// vectors are rhs-inner [site][comp][rhs], so a B operand is 16 contiguous RHS.
// FP16S links (one fp32 scale per coarse site and link) use
// v_mfma_f32_16x16x16_f16 with fp32 accumulation, the scale applied per link.
#include "coarse.h"
#include "field.h"

namespace crk {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx4 __attribute__((ext_vector_type(4)));

template <class T> struct Mfma;
template <> struct Mfma<float> {
  using acc = floatx4;
  __device__ static __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  using acc = doublex4;
  __device__ static __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// One workgroup of three wavefronts per (coarse site, 16-RHS tile, 16-row
// tile); wavefront w accumulates links 3w .. 3w+2 (X and the eight hops), the
// partial tiles are added in LDS in a fixed order.  2k/16 row tiles of one site
// and RHS tile share the B operands through the cache; splitting the nine
// links gives the small coarse lattices enough wavefronts to keep loads in
// flight.
constexpr int kLinkWaves = 3;
constexpr int kLinksPerWave = 9 / kLinkWaves;

template <class T, int MT>
__global__ __launch_bounds__(64 * kLinkWaves) void coarse_mfma_kernel(const typename cplx_t<T>::type* __restrict__ links,
                                                                      const typename cplx_t<T>::type* __restrict__ in,
                                                                      typename cplx_t<T>::type* __restrict__ out,
                                                                      const int* __restrict__ nbr, int64_t Vc, int nrhs,
                                                                      int ntiles, T sign,
                                                                      typename cplx_t<T>::type* __restrict__ copy) {
  using C = typename cplx_t<T>::type;
  using A = typename Mfma<T>::acc;
  constexpr int N = 16 * MT;
  __shared__ T part[kLinkWaves - 1][8][64];
  const int mt = blockIdx.x % MT;
  const int64_t rest = blockIdx.x / MT;
  const int tile = int(rest % ntiles);
  const int64_t j = rest / ntiles;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n = tile * 16 + (lane & 15);
  const int kq = lane >> 4;
  const bool live = n < nrhs;
  // columns past nrhs read the last RHS (in bounds, no branch around the loads,
  // so the loads of all K steps can be in flight together); output column n of
  // a product depends on B column n only, and those columns are not stored
  const int nc = live ? n : nrhs - 1;
  // The wavefront's three links: the A and B operands of link t + 1 are loaded
  // while link t is multiplied; two accumulators per real/imaginary part keep
  // consecutive MFMAs independent.
  constexpr int KS = N / 4;
  A are0 = A{0, 0, 0, 0}, are1 = A{0, 0, 0, 0}, aim0 = A{0, 0, 0, 0}, aim1 = A{0, 0, 0, 0};
  C av[KS], bv[KS];
  auto load_link = [&](int nb, C (&a)[KS], C (&b)[KS]) {
    const int64_t s = nb == 0 ? j : int64_t(nbr[int64_t(nb - 1) * Vc + j]);
    const C* Lb = links + (j * 9 + nb) * int64_t(N) * N + mt * 16 + (lane & 15);
    const C* vb = in + s * int64_t(N) * nrhs + nc;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int kk = ks * 4 + kq;
      a[ks] = Lb[int64_t(kk) * N];
      b[ks] = vb[int64_t(kk) * nrhs];
    }
  };
  load_link(kLinksPerWave * wv, av, bv);
#pragma unroll
  for (int t = 0; t < kLinksPerWave; ++t) {
    C an[KS], bn[KS];
    if (t + 1 < kLinksPerWave) load_link(kLinksPerWave * wv + t + 1, an, bn);
    // keep the next link's loads above this link's products (the scheduler
    // would otherwise sink each load to its use and wait on it there)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      are0 = Mfma<T>::op(av[ks].x, bv[ks].x, are0);
      aim0 = Mfma<T>::op(av[ks].x, bv[ks].y, aim0);
      are1 = Mfma<T>::op(-av[ks].y, bv[ks].y, are1);
      aim1 = Mfma<T>::op(av[ks].y, bv[ks].x, aim1);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (t + 1 < kLinksPerWave) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        av[ks] = an[ks];
        bv[ks] = bn[ks];
      }
    }
  }
  A are, aim;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    are[i] = are0[i] + are1[i];
    aim[i] = aim0[i] + aim1[i];
  }
  if (wv > 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      part[wv - 1][i][lane] = are[i];
      part[wv - 1][4 + i][lane] = aim[i];
    }
  }
  __syncthreads();
  if (wv > 0 || !live) return;
  if (copy) {  // copy of the input rows of this tile (lets a caller keep z = in without a copy launch)
    const C* vin = in + j * int64_t(N) * nrhs + n;
    C* vc = copy + j * int64_t(N) * nrhs + n;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = mt * 16 + kq * 4 + i;
      vc[int64_t(row) * nrhs] = vin[int64_t(row) * nrhs];
    }
  }
#pragma unroll
  for (int w = 0; w < kLinkWaves - 1; ++w)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      are[i] += part[w][i][lane];
      aim[i] += part[w][4 + i][lane];
    }
  C* ob = out + j * int64_t(N) * nrhs + n;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    // accumulator layout: f32 16x16x4 holds rows 4*(lane/16) + i, f64 16x16x4 rows lane/16 + 4*i
    const int row = mt * 16 + (sizeof(T) == 8 ? kq + 4 * i : kq * 4 + i);
    ob[int64_t(row) * nrhs] = C{sign * are[i], sign * aim[i]};
  }
}

// FP16 links with a per-(site, link) fp32 scale; fp32 vectors; fp32 accumulation.
// A operand of 16x16x16f16: lane holds A[row = lane%16][k = 4*(lane/16) + i], i < 4.
// One workgroup of nine wavefronts per (coarse site, 16-RHS tile): wavefront nb
// takes link nb for all 2k/16 row tiles.  Per link the B operand (the
// neighbour's vector column) is scaled by its largest entry so that it is well
// conditioned in fp16, and the product is rescaled by that value and the
// link's scale in fp32; the nine rescaled products are then added in link
// order through LDS.
constexpr int kF16Waves = 9;

template <int MT>
__global__ __launch_bounds__(64 * kF16Waves) void coarse_mfma_f16_kernel(const __half2* __restrict__ links,
                                                                         const float* __restrict__ lscale,
                                                                         const float2* __restrict__ in,
                                                                         float2* __restrict__ out,
                                                                         const int* __restrict__ nbr, int64_t Vc,
                                                                         int nrhs, int ntiles, float sign,
                                                                         float2* __restrict__ copy) {
  constexpr int N = 16 * MT;
  __shared__ float part[kF16Waves - 1][MT][8][64];
  const int64_t j = blockIdx.x / ntiles;
  const int tile = blockIdx.x % ntiles;
  const int lane = threadIdx.x & 63, nb = threadIdx.x >> 6;
  const int n = tile * 16 + (lane & 15);
  const int kq = lane >> 4;
  const bool live = n < nrhs;
  const int nc = live ? n : nrhs - 1;  // past nrhs: the last RHS (in bounds), not stored
  const int64_t s = nb == 0 ? j : int64_t(nbr[int64_t(nb - 1) * Vc + j]);
  const __half2* Lb = links + (j * 9 + nb) * int64_t(N) * N + (lane & 15);
  const float2* vb = in + s * int64_t(N) * nrhs + nc;
  const float ls = lscale[j * 9 + nb];
  float vmax = 0.f;
#pragma unroll
  for (int kk = 0; kk < N; ++kk) {
    const float2 v = vb[int64_t(kk) * nrhs];
    vmax = fmaxf(vmax, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  const float vinv = vmax > 0.f ? 1.f / vmax : 0.f;
  floatx4 are[MT], aim[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) { are[mt] = floatx4{0, 0, 0, 0}; aim[mt] = floatx4{0, 0, 0, 0}; }
#pragma unroll
  for (int ks = 0; ks < N / 16; ++ks) {
    halfx4 br, bi;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float2 v = vb[int64_t(ks * 16 + kq * 4 + i) * nrhs];
      br[i] = _Float16(v.x * vinv);
      bi[i] = _Float16(v.y * vinv);
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      halfx4 ar, ai, ain;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const __half2 a = Lb[int64_t(ks * 16 + kq * 4 + i) * N + mt * 16];
        ar[i] = __builtin_bit_cast(_Float16, a.x);
        ai[i] = __builtin_bit_cast(_Float16, a.y);
        ain[i] = -ai[i];
      }
      are[mt] = __builtin_amdgcn_mfma_f32_16x16x16f16(ar, br, are[mt], 0, 0, 0);
      are[mt] = __builtin_amdgcn_mfma_f32_16x16x16f16(ain, bi, are[mt], 0, 0, 0);
      aim[mt] = __builtin_amdgcn_mfma_f32_16x16x16f16(ar, bi, aim[mt], 0, 0, 0);
      aim[mt] = __builtin_amdgcn_mfma_f32_16x16x16f16(ai, br, aim[mt], 0, 0, 0);
    }
  }
  // the lane's output column n has the same vector scale for every row
  const float f = ls * vmax;
  if (nb > 0) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        part[nb - 1][mt][i][lane] = f * are[mt][i];
        part[nb - 1][mt][4 + i][lane] = f * aim[mt][i];
      }
  }
  __syncthreads();
  if (nb > 0 || !live) return;
  float2* ob = out + j * int64_t(N) * nrhs + n;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    floatx4 tre, tim;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      tre[i] = 0.f + f * are[mt][i];
      tim[i] = 0.f + f * aim[mt][i];
    }
#pragma unroll
    for (int w = 0; w < kF16Waves - 1; ++w)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        tre[i] += part[w][mt][i][lane];
        tim[i] += part[w][mt][4 + i][lane];
      }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = mt * 16 + kq * 4 + i;
      ob[int64_t(row) * nrhs] = float2{sign * tre[i], sign * tim[i]};
    }
  }
  if (copy) {
    const float2* vin = in + j * int64_t(N) * nrhs + n;
    float2* vc = copy + j * int64_t(N) * nrhs + n;
#pragma unroll
    for (int row = kq * 4; row < N; row += 16)
#pragma unroll
      for (int i = 0; i < 4; ++i) vc[int64_t(row + i) * nrhs] = vin[int64_t(row + i) * nrhs];
  }
}

__global__ void links_to_f32_kernel(const double2* __restrict__ src, float2* __restrict__ dst, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = make_float2(float(src[i].x), float(src[i].y));
}

// One workgroup per (site, link) block: scale = max |re|, |im| of the block.
__global__ __launch_bounds__(256) void links_to_f16_kernel(const double2* __restrict__ src, __half2* __restrict__ dst,
                                                           float* __restrict__ scale, int N) {
  __shared__ float red[256];
  const int64_t b = blockIdx.x;
  const double2* s = src + b * int64_t(N) * N;
  float m = 0.f;
  for (int e = threadIdx.x; e < N * N; e += blockDim.x)
    m = fmaxf(m, fmaxf(float(fabs(s[e].x)), float(fabs(s[e].y))));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  const float mx = red[0];
  const float inv = mx > 0.f ? 1.f / mx : 0.f;
  if (threadIdx.x == 0) scale[b] = mx;
  for (int e = threadIdx.x; e < N * N; e += blockDim.x)
    dst[b * int64_t(N) * N + e] = __floats2half2_rn(float(s[e].x) * inv, float(s[e].y) * inv);
}

template <class T>
void launch_mfma(int N, const void* links, const void* in, void* out, const int* nbr, int64_t Vc, int nrhs, T sign,
                 void* copy, hipStream_t st) {
  using C = typename cplx_t<T>::type;
  CRK_REQUIRE(N % 16 == 0 && N >= 16 && N <= 64, "coarse operator: 2k must be 16, 32, 48 or 64");
  const int ntiles = (nrhs + 15) / 16;
  const dim3 g = dim3(unsigned(Vc * ntiles * (N / 16)));
  const dim3 b(64 * kLinkWaves);
  const C* L = static_cast<const C*>(links);
  const C* x = static_cast<const C*>(in);
  C* y = static_cast<C*>(out);
  C* cp = static_cast<C*>(copy);
  switch (N / 16) {
    case 1: hipLaunchKernelGGL((coarse_mfma_kernel<T, 1>), g, b, 0, st, L, x, y, nbr, Vc, nrhs, ntiles, sign, cp); break;
    case 2: hipLaunchKernelGGL((coarse_mfma_kernel<T, 2>), g, b, 0, st, L, x, y, nbr, Vc, nrhs, ntiles, sign, cp); break;
    case 3: hipLaunchKernelGGL((coarse_mfma_kernel<T, 3>), g, b, 0, st, L, x, y, nbr, Vc, nrhs, ntiles, sign, cp); break;
    default: hipLaunchKernelGGL((coarse_mfma_kernel<T, 4>), g, b, 0, st, L, x, y, nbr, Vc, nrhs, ntiles, sign, cp); break;
  }
  CRK_LAUNCH_CHECK();
}

void launch_f16(int N, const void* links, const void* in, void* out, const int* nbr, int64_t Vc, int nrhs, float sign,
                void* copy, hipStream_t st) {
  const int ntiles = (nrhs + 15) / 16;
  const dim3 g = dim3(unsigned(Vc * ntiles));
  const dim3 b(64 * kF16Waves);
  const __half2* L = static_cast<const __half2*>(links);
  const float* ls = reinterpret_cast<const float*>(L + Vc * 9 * int64_t(N) * N);
  const float2* x = static_cast<const float2*>(in);
  float2* y = static_cast<float2*>(out);
  float2* cp = static_cast<float2*>(copy);
  switch (N / 16) {
    case 1: hipLaunchKernelGGL((coarse_mfma_f16_kernel<1>), g, b, 0, st, L, ls, x, y, nbr, Vc, nrhs, ntiles, sign, cp); break;
    case 2: hipLaunchKernelGGL((coarse_mfma_f16_kernel<2>), g, b, 0, st, L, ls, x, y, nbr, Vc, nrhs, ntiles, sign, cp); break;
    case 3: hipLaunchKernelGGL((coarse_mfma_f16_kernel<3>), g, b, 0, st, L, ls, x, y, nbr, Vc, nrhs, ntiles, sign, cp); break;
    case 4: hipLaunchKernelGGL((coarse_mfma_f16_kernel<4>), g, b, 0, st, L, ls, x, y, nbr, Vc, nrhs, ntiles, sign, cp); break;
    default: fail(CRK_EINVAL, "coarse operator: 2k must be 16, 32, 48 or 64");
  }
  CRK_LAUNCH_CHECK();
}

}  // namespace

size_t coarse_links_bytes(int form, int64_t Vc, int N) {
  const size_t n = size_t(Vc) * 9 * N * N;
  if (form == CRK_FORM_FP64) return n * sizeof(double2);
  if (form == CRK_FORM_FP32) return n * sizeof(float2);
  return n * sizeof(__half2) + size_t(Vc) * 9 * sizeof(float);
}

void coarse_links_convert(const void* links64, int form, void* dst, int64_t Vc, int N, hipStream_t st) {
  const int64_t n = Vc * 9 * int64_t(N) * N;
  if (form == CRK_FORM_FP32) {
    hipLaunchKernelGGL(links_to_f32_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st,
                       static_cast<const double2*>(links64), static_cast<float2*>(dst), n);
  } else if (form == CRK_FORM_FP16S) {
    __half2* h = static_cast<__half2*>(dst);
    float* sc = reinterpret_cast<float*>(h + n);
    hipLaunchKernelGGL(links_to_f16_kernel, dim3(unsigned(Vc * 9)), dim3(256), 0, st,
                       static_cast<const double2*>(links64), h, sc, N);
  } else {
    fail(CRK_EINVAL, "coarse_links_convert: target form must be FP32 or FP16S");
  }
  CRK_LAUNCH_CHECK();
}

void coarse_apply(int form, int N, const void* links, const void* in, void* out, const int* nbr, int64_t Vc, int nrhs,
                  bool negate, hipStream_t st, void* copy) {
  if (nrhs <= 0 || Vc <= 0) return;
  CRK_REQUIRE(in != out && copy != out && copy != in, "coarse apply: in, out and copy must not alias");
  if (form == CRK_FORM_FP64) launch_mfma<double>(N, links, in, out, nbr, Vc, nrhs, negate ? -1.0 : 1.0, copy, st);
  else if (form == CRK_FORM_FP32) launch_mfma<float>(N, links, in, out, nbr, Vc, nrhs, negate ? -1.f : 1.f, copy, st);
  else launch_f16(N, links, in, out, nbr, Vc, nrhs, negate ? -1.f : 1.f, copy, st);
}

}  // namespace crk
