// Multi-RHS Wilson-Dirac operator on the fine lattice.
//
// D psi(x) = (m0 + sum_mu w_mu) psi(x)
//          - 1/2 sum_mu w_mu [(1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)]
// in the chiral basis (gamma5 = diag(1,1,-1,-1)), w = (1,1,1,1/xi).
//
// Each (1 -+ gamma_mu) has rank 2, so every hop projects the neighbour spinor
// to a half spinor (2 spins x 3 colours), multiplies by the SU(3) link and
// rebuilds the lower spins from the upper ones.  Neighbour addresses come
// from a per-site table, so any site order (lexicographic or block-major) can
// be served.  Kernels: wilson_tile_kernel (the fine level of a hierarchy with
// 4^4 blocks, FP32 and FP16 storage: a block and its faces staged in LDS),
// wilson_rhsloop_kernel (FP32, any order: one thread per site, links in
// registers across the RHS loop), wilson_dir_kernel (FP64: one wavefront per
// direction, partial spinors exchanged through LDS) and wilson_kernel<FORM, R>
// (R right-hand sides per thread, the remaining cases).  Optionally a launch
// also emits per-wavefront partial sums <Dr, r> and <Dr, Dr> for the
// minimal-residual smoother, so no separate pass over the fields is needed.
#include "field.h"
#include "kernels.h"

namespace crk {

namespace {

constexpr int kDirMaxRhs = 64;  // right-hand sides of one direction-split launch (partial sums in LDS)

// Spin projection of psi onto the half spinor of (1 - sign*gamma_mu).
template <int MU, int SIGN, class C>
__device__ __forceinline__ void project(const C* s, C* h) {
  // s[3*spin + colour]
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    C s0 = s[a], s1 = s[3 + a], s2 = s[6 + a], s3 = s[9 + a];
    if constexpr (MU == 0) {
      if constexpr (SIGN > 0) { h[a] = s0 + cmuli(s3); h[3 + a] = s1 + cmuli(s2); }
      else { h[a] = s0 - cmuli(s3); h[3 + a] = s1 - cmuli(s2); }
    } else if constexpr (MU == 1) {
      if constexpr (SIGN > 0) { h[a] = s0 + s3; h[3 + a] = s1 - s2; }
      else { h[a] = s0 - s3; h[3 + a] = s1 + s2; }
    } else if constexpr (MU == 2) {
      if constexpr (SIGN > 0) { h[a] = s0 + cmuli(s2); h[3 + a] = s1 - cmuli(s3); }
      else { h[a] = s0 - cmuli(s2); h[3 + a] = s1 + cmuli(s3); }
    } else {
      if constexpr (SIGN > 0) { h[a] = s0 - s2; h[3 + a] = s1 - s3; }
      else { h[a] = s0 + s2; h[3 + a] = s1 + s3; }
    }
  }
}

// acc += coef * (full spinor rebuilt from the link-multiplied half spinor g).
template <int MU, int SIGN, class C, class T>
__device__ __forceinline__ void accumulate(C* acc, const C* g, T coef) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    C g0 = g[a], g1 = g[3 + a];
    C l2, l3;
    if constexpr (MU == 0) {
      if constexpr (SIGN > 0) { l2 = cscale(cmuli(g1), T(-1)); l3 = cscale(cmuli(g0), T(-1)); }
      else { l2 = cmuli(g1); l3 = cmuli(g0); }
    } else if constexpr (MU == 1) {
      if constexpr (SIGN > 0) { l2 = cscale(g1, T(-1)); l3 = g0; }
      else { l2 = g1; l3 = cscale(g0, T(-1)); }
    } else if constexpr (MU == 2) {
      if constexpr (SIGN > 0) { l2 = cscale(cmuli(g0), T(-1)); l3 = cmuli(g1); }
      else { l2 = cmuli(g0); l3 = cscale(cmuli(g1), T(-1)); }
    } else {
      if constexpr (SIGN > 0) { l2 = cscale(g0, T(-1)); l3 = cscale(g1, T(-1)); }
      else { l2 = g0; l3 = g1; }
    }
    acc[a].x = fma(coef, g0.x, acc[a].x);     acc[a].y = fma(coef, g0.y, acc[a].y);
    acc[3 + a].x = fma(coef, g1.x, acc[3 + a].x); acc[3 + a].y = fma(coef, g1.y, acc[3 + a].y);
    acc[6 + a].x = fma(coef, l2.x, acc[6 + a].x); acc[6 + a].y = fma(coef, l2.y, acc[6 + a].y);
    acc[9 + a].x = fma(coef, l3.x, acc[9 + a].x); acc[9 + a].y = fma(coef, l3.y, acc[9 + a].y);
  }
}

// g = U h (forward) or U^dag h (backward), per half-spin.
template <int SIGN, class C>
__device__ __forceinline__ void link_mul(const C* u, const C* h, C* g) {
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      C t = czero<C>();
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if constexpr (SIGN > 0) cfma(t, u[3 * a + b], h[3 * sp + b]);
        else cfmac(t, u[3 * b + a], h[3 * sp + b]);
      }
      g[3 * sp + a] = t;
    }
  }
}

// Clover site term (Wilson-clover operator): acc = sign * X(s) psi with X the
// two 6 x 6 chirality blocks of site s (diagonal included), stored
// site-vectorised with 72 components, entry 36*alpha + 6*r + c.
template <class S, class C, class T>
__device__ __forceinline__ void clover_site(const S* __restrict__ cl, int64_t Vp, int64_t s, const C (&psi)[12],
                                            C (&acc)[12], T sign) {
  const S* p = cl + aidx(0, 0, s, Vp, 72);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      C t = czero<C>();
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const S x = p[(36 * a + 6 * r + c) * kVL];
        cfma(t, mk<C>(x.x, x.y), psi[6 * a + c]);
      }
      acc[6 * a + r] = cscale(t, sign);
      // one row's six loads at a time: the kernels that call this already hold
      // their links in registers, and hoisting all 72 loads would spill them
      asm volatile("" ::: "memory");
    }
}

template <int FORM, int R, int MU, int SIGN>
__device__ __forceinline__ void hop(const FineView<FORM>& in, const GaugeView<FORM>& U, const int* __restrict__ nbr,
                                    int64_t V, int64_t s, int r0, int nrhs,
                                    typename Prec<FORM>::cx (&acc)[R][12], typename Prec<FORM>::real coef) {
  using C = typename Prec<FORM>::cx;
  const int64_t y = nbr[int64_t(2 * MU + (SIGN > 0 ? 0 : 1)) * V + s];
  C u[9];
  U.load(MU, SIGN > 0 ? s : y, u);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r0 + r < nrhs) {
      C psi[12], h[6], g[6];
      in.load(r0 + r, y, psi);
      project<MU, SIGN>(psi, h);
      link_mul<SIGN>(u, h, g);
      accumulate<MU, SIGN>(acc[r], g, coef);
    }
  }
}

template <int FORM, int R, bool CL>
__global__ __launch_bounds__(256) void wilson_kernel(FineView<FORM> in, FineView<FORM> out, GaugeView<FORM> U,
                                                     const int* __restrict__ nbr, int64_t V, int nrhs, int ngroups,
                                                     typename Prec<FORM>::real diag, float4 hw_f, double4 hw_d,
                                                     double* __restrict__ partial, int64_t nsb, int order,
                                                     int swz, const void* __restrict__ clv,
                                                     typename Prec<FORM>::real csign) {
  using C = typename Prec<FORM>::cx;
  using T = typename Prec<FORM>::real;
  const uint32_t L = swz ? xcd_swizzle(blockIdx.x, gridDim.x) : blockIdx.x;
  // order 0: the RHS groups of one site block are consecutive (links reused in L2);
  // order 1: all site blocks of one RHS group are consecutive (halos reused in L2)
  const int64_t sb = order == 0 ? L / ngroups : L % nsb;
  const int g = order == 0 ? int(L % ngroups) : int(L / nsb);
  const int64_t s = sb * blockDim.x + threadIdx.x;
  const int r0 = g * R;
  const bool live = s < V;
  T hw[4];
  if constexpr (FORM == CRK_FORM_FP64) { hw[0] = hw_d.x; hw[1] = hw_d.y; hw[2] = hw_d.z; hw[3] = hw_d.w; }
  else { hw[0] = hw_f.x; hw[1] = hw_f.y; hw[2] = hw_f.z; hw[3] = hw_f.w; }

  C acc[R][12];
  double dqr_re[R], dqr_im[R], dqq[R];
  if (live) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r0 + r < nrhs) {
        C psi[12];
        in.load(r0 + r, s, psi);
        if constexpr (CL) {
          clover_site(static_cast<const typename Prec<FORM>::cx*>(clv), in.Vp, s, psi, acc[r], csign);
        } else {
#pragma unroll
          for (int c = 0; c < 12; ++c) acc[r][c] = cscale(psi[c], diag);
        }
      } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[r][c] = czero<C>();
      }
    }
    hop<FORM, R, 0, +1>(in, U, nbr, V, s, r0, nrhs, acc, hw[0]);
    hop<FORM, R, 0, -1>(in, U, nbr, V, s, r0, nrhs, acc, hw[0]);
    hop<FORM, R, 1, +1>(in, U, nbr, V, s, r0, nrhs, acc, hw[1]);
    hop<FORM, R, 1, -1>(in, U, nbr, V, s, r0, nrhs, acc, hw[1]);
    hop<FORM, R, 2, +1>(in, U, nbr, V, s, r0, nrhs, acc, hw[2]);
    hop<FORM, R, 2, -1>(in, U, nbr, V, s, r0, nrhs, acc, hw[2]);
    hop<FORM, R, 3, +1>(in, U, nbr, V, s, r0, nrhs, acc, hw[3]);
    hop<FORM, R, 3, -1>(in, U, nbr, V, s, r0, nrhs, acc, hw[3]);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r0 + r < nrhs) out.store(r0 + r, s, acc[r]);
  }
  if (partial == nullptr) return;
  // <q, r> and <q, q> with q = D r (this output) and r = the input at s.
#pragma unroll
  for (int r = 0; r < R; ++r) {
    dqr_re[r] = dqr_im[r] = dqq[r] = 0.0;
    if (live && r0 + r < nrhs) {
      C psi[12];
      in.load(r0 + r, s, psi);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const C q = acc[r][c];
        dqr_re[r] += double(q.x) * psi[c].x + double(q.y) * psi[c].y;
        dqr_im[r] += double(q.x) * psi[c].y - double(q.y) * psi[c].x;
        dqq[r] += double(q.x) * q.x + double(q.y) * q.y;
      }
    }
  }
  // one partial row per wavefront (64 sites): no workgroup reduction needed
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double v0 = dqr_re[r], v1 = dqr_im[r], v2 = dqq[r];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      v0 += __shfl_xor(v0, o);
      v1 += __shfl_xor(v1, o);
      v2 += __shfl_xor(v2, o);
    }
    if (lane == 0 && r0 + r < nrhs && (sb * 4 + wid) * kVL < V) {
      double* p = partial + ((sb * 4 + wid) * nrhs + (r0 + r)) * 3;
      p[0] = v0;
      p[1] = v1;
      p[2] = v2;
    }
  }
}

// Variant that keeps the eight links of a site in registers and loops over all
// right-hand sides inside the thread.  Links are read from memory once per
// site instead of once per RHS group, and since every workgroup of the grid
// walks the RHS in the same order, the workgroups resident on one XCD touch
// the same RHS at the same time: the neighbour (halo) spinors they share are
// then reused from that XCD's L2 instead of being fetched again.
template <int FORM, int MU, int SIGN>
__device__ __forceinline__ void hop_reg(const FineView<FORM>& in, int64_t r, int64_t y,
                                        const typename GaugeView<FORM>::S (&u)[9],
                                        typename Prec<FORM>::cx (&acc)[12], typename Prec<FORM>::real coef) {
  using C = typename Prec<FORM>::cx;
  C uc[9], psi[12], h[6], g[6];
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    if constexpr (FORM == CRK_FORM_FP16S) uc[e] = __half22float2(u[e]);
    else uc[e] = u[e];
  }
  in.load(r, y, psi);
  project<MU, SIGN>(psi, h);
  link_mul<SIGN>(uc, h, g);
  accumulate<MU, SIGN>(acc, g, coef);
}

template <int FORM, bool CL>
__global__ __launch_bounds__(256) void wilson_rhsloop_kernel(FineView<FORM> in, FineView<FORM> out, GaugeView<FORM> U,
                                                             const int* __restrict__ nbr, int64_t V, int nrhs,
                                                             typename Prec<FORM>::real diag, float4 hw,
                                                             double* __restrict__ partial, int swz,
                                                             const void* __restrict__ clv,
                                                             typename Prec<FORM>::real csign) {
  using C = typename Prec<FORM>::cx;
  using T = typename Prec<FORM>::real;
  using S = typename GaugeView<FORM>::S;
  const int64_t sb = swz ? xcd_swizzle(blockIdx.x, gridDim.x) : blockIdx.x;
  const int64_t s = sb * blockDim.x + threadIdx.x;
  const bool live = s < V;
  const int64_t sl = live ? s : 0;  // dead lanes compute on site 0 and store nothing
  int y[8];
  S u[8][9];
#pragma unroll
  for (int d = 0; d < 8; ++d) y[d] = nbr[int64_t(d) * V + sl];
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    const S* p = U.data + aidx(d >> 1, 0, (d & 1) ? int64_t(y[d]) : sl, U.Vp, 9);
#pragma unroll
    for (int e = 0; e < 9; ++e) u[d][e] = p[e * kVL];
  }
  const T hw0 = hw.x, hw1 = hw.y, hw2 = hw.z, hw3 = hw.w;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int r = 0; r < nrhs; ++r) {
    C acc[12];
    {
      C psi[12];
      in.load(r, sl, psi);
      if constexpr (CL) {
        clover_site(static_cast<const typename Prec<FORM>::cx*>(clv), in.Vp, sl, psi, acc, csign);
      } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = cscale(psi[c], diag);
      }
    }
    hop_reg<FORM, 0, +1>(in, r, y[0], u[0], acc, hw0);
    hop_reg<FORM, 0, -1>(in, r, y[1], u[1], acc, hw0);
    hop_reg<FORM, 1, +1>(in, r, y[2], u[2], acc, hw1);
    hop_reg<FORM, 1, -1>(in, r, y[3], u[3], acc, hw1);
    hop_reg<FORM, 2, +1>(in, r, y[4], u[4], acc, hw2);
    hop_reg<FORM, 2, -1>(in, r, y[5], u[5], acc, hw2);
    hop_reg<FORM, 3, +1>(in, r, y[6], u[6], acc, hw3);
    hop_reg<FORM, 3, -1>(in, r, y[7], u[7], acc, hw3);
    if (live) out.store(r, s, acc);
    if (partial != nullptr) {
      double v0 = 0, v1 = 0, v2 = 0;
      if (live) {
        C psi[12];
        in.load(r, s, psi);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const C q = acc[c];
          v0 += double(q.x) * psi[c].x + double(q.y) * psi[c].y;
          v1 += double(q.x) * psi[c].y - double(q.y) * psi[c].x;
          v2 += double(q.x) * q.x + double(q.y) * q.y;
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        v0 += __shfl_xor(v0, o);
        v1 += __shfl_xor(v1, o);
        v2 += __shfl_xor(v2, o);
      }
      // one partial row per wavefront (64 sites)
      if (lane == 0 && (sb * 4 + wid) * kVL < V) {
        double* p = partial + ((sb * 4 + wid) * nrhs + r) * 3;
        p[0] = v0;
        p[1] = v1;
        p[2] = v2;
      }
    }
  }
}

template <int FORM>
void launch_wilson_rhsloop(const WilsonArgs& a, hipStream_t st) {
  const int64_t nsb = (a.V + 255) / 256;
  FineView<FORM> in(const_cast<void*>(a.in), a.V, a.nrhs), out(a.out, a.V, a.nrhs);
  GaugeView<FORM> U{static_cast<const typename Prec<FORM>::store*>(a.gauge), pad_sites(a.V)};
  const float4 hw = make_float4(float(a.hw[0]), float(a.hw[1]), float(a.hw[2]), float(a.hw[3]));
  if (a.clover)
    hipLaunchKernelGGL((wilson_rhsloop_kernel<FORM, true>), dim3(unsigned(nsb)), dim3(256), 0, st, in, out, U, a.nbr,
                       a.V, a.nrhs, typename Prec<FORM>::real(a.diag), hw, a.partial, a.swizzle, a.clover,
                       typename Prec<FORM>::real(a.clover_sign));
  else
    hipLaunchKernelGGL((wilson_rhsloop_kernel<FORM, false>), dim3(unsigned(nsb)), dim3(256), 0, st, in, out, U, a.nbr,
                       a.V, a.nrhs, typename Prec<FORM>::real(a.diag), hw, a.partial, a.swizzle, a.clover,
                       typename Prec<FORM>::real(a.clover_sign));
  CRK_LAUNCH_CHECK();
}

// One complex entry of input storage FIN in the arithmetic type C (FP32
// storage read by the FP64 operator: widened exactly).
template <class C, class S> __device__ __forceinline__ C widen(const S& v) { return mk<C>(v.x, v.y); }

// Spinor of site y, RHS r, of an input in storage FIN, in the arithmetic of FORM.
template <int FORM, int FIN>
__device__ __forceinline__ void load_as(const FineView<FIN>& in, int64_t r, int64_t y,
                                        typename Prec<FORM>::cx (&v)[12]) {
  if constexpr (FIN == FORM) {
    in.load(r, y, v);
  } else {
    typename Prec<FIN>::cx raw[12];
    in.load(r, y, raw);
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = widen<typename Prec<FORM>::cx>(raw[c]);
  }
}

// Both hops along MU for one RHS: the spin-MU components of the partial result
// are returned in m0, m1, m2 (three scalars, not an array: an array written in
// the four branches of the caller's switch was kept on the stack), the other
// nine go to their owners' exchange slots.
template <int FORM, int FIN, int MU>
__device__ __forceinline__ void hop_pair(const FineView<FIN>& in, int r, int64_t yf, int64_t yb,
                                         const typename Prec<FORM>::cx (&uf)[9],
                                         const typename Prec<FORM>::cx (&ub)[9], typename Prec<FORM>::real coef,
                                         typename Prec<FORM>::cx (*xch)[3][kVL], int lane,
                                         typename Prec<FORM>::cx& m0, typename Prec<FORM>::cx& m1,
                                         typename Prec<FORM>::cx& m2) {
  using C = typename Prec<FORM>::cx;
  C acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = czero<C>();
  C psi[12], h[6], g[6];
  load_as<FORM, FIN>(in, r, yf, psi);
  project<MU, +1>(psi, h);
  link_mul<+1>(uf, h, g);
  accumulate<MU, +1>(acc, g, coef);
  load_as<FORM, FIN>(in, r, yb, psi);
  project<MU, -1>(psi, h);
  link_mul<-1>(ub, h, g);
  accumulate<MU, -1>(acc, g, coef);
#pragma unroll
  for (int o = 0; o < 4; ++o) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (o == MU) {
        if (c == 0) m0 = acc[3 * o];
        else if (c == 1) m1 = acc[3 * o + 1];
        else m2 = acc[3 * o + 2];
      }
      else xch[3 * MU + (o < MU ? o : o - 1)][c][lane] = acc[3 * o + c];
    }
  }
}

// Direction-split variant: a workgroup covers 64 sites with four wavefronts,
// wavefront mu handling the two hops along mu for all 64 sites.  Its two
// links stay in registers for the whole right-hand-side loop (18 complex per
// thread instead of 72), which keeps several wavefronts per SIMD in flight.
// Per RHS wavefront mu keeps the three components of spin mu of its partial
// result and hands the other nine to their owners through LDS; after a barrier
// it adds the diagonal term and the four partials of spin mu in a fixed order
// and stores them.  A second barrier frees the LDS slots for the next RHS.
// FIN is the storage of the input: FORM itself, or FP32 for the FP64 operator
// applied to a field that holds FP32 values (the outer solver's directions in
// the reduced-precision forms), read as such and widened exactly.
template <int FORM, int FIN, bool CL>
__global__ __launch_bounds__(256) void wilson_dir_kernel(FineView<FIN> in, FineView<FORM> out, GaugeView<FORM> U,
                                                         const int* __restrict__ nbr, int64_t V, int nrhs,
                                                         typename Prec<FORM>::real diag, double4 hw_d,
                                                         double* __restrict__ partial, int swz,
                                                         const void* __restrict__ clv,
                                                         typename Prec<FORM>::real csign) {
  using C = typename Prec<FORM>::cx;
  using T = typename Prec<FORM>::real;
  using S = typename Prec<FORM>::store;
  using SI = typename Prec<FIN>::store;
  // xch[3*src + slot][c][site]: spin `owner` components of wavefront src's partial,
  // slot = owner with src skipped (owner != src)
  __shared__ C xch[12][3][kVL];
  __shared__ double red[4][kDirMaxRhs][3];
  const int64_t blk = swz ? xcd_swizzle(blockIdx.x, gridDim.x) : blockIdx.x;
  const int mu = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t s = blk * kVL + lane;
  const bool live = s < V;
  const int64_t sl = live ? s : 0;  // dead lanes compute on site 0 and store nothing
  const int64_t yf = nbr[int64_t(2 * mu) * V + sl], yb = nbr[int64_t(2 * mu + 1) * V + sl];
  C uf[9], ub[9];
  {
    const S* pf = U.data + aidx(mu, 0, sl, U.Vp, 9);
    const S* pb = U.data + aidx(mu, 0, yb, U.Vp, 9);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      uf[e] = pf[e * kVL];
      ub[e] = pb[e * kVL];
    }
  }
  const T coef = T(mu == 0 ? hw_d.x : mu == 1 ? hw_d.y : mu == 2 ? hw_d.z : hw_d.w);
  for (int r = 0; r < nrhs; ++r) {
    C m0, m1, m2;
    switch (mu) {
      case 0: hop_pair<FORM, FIN, 0>(in, r, yf, yb, uf, ub, coef, xch, lane, m0, m1, m2); break;
      case 1: hop_pair<FORM, FIN, 1>(in, r, yf, yb, uf, ub, coef, xch, lane, m0, m1, m2); break;
      case 2: hop_pair<FORM, FIN, 2>(in, r, yf, yb, uf, ub, coef, xch, lane, m0, m1, m2); break;
      default: hop_pair<FORM, FIN, 3>(in, r, yf, yb, uf, ub, coef, xch, lane, m0, m1, m2); break;
    }
    __syncthreads();
    // spin mu of site s: diagonal + the partials of wavefronts 0..3 (fixed order)
    const SI* pin = in.data + aidx(r, 3 * mu, sl, in.Vp, 12);
    S* pout = out.data + aidx(r, 3 * mu, sl, out.Vp, 12);
    double v0 = 0, v1 = 0, v2 = 0;
    C site[3];
    if constexpr (CL) {
      // rows 3 (mu % 2) + c of the chirality-(mu / 2) clover block times that chirality's six components
      const int al = mu >> 1, r0 = 3 * (mu & 1);
      const SI* pc = in.data + aidx(r, 6 * al, sl, in.Vp, 12);
      const C* X = static_cast<const C*>(clv) + aidx(0, 36 * al + 6 * r0, sl, in.Vp, 72);
      C ps[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) ps[j] = widen<C>(pc[j * kVL]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        C t = czero<C>();
#pragma unroll
        for (int j = 0; j < 6; ++j) cfma(t, X[(6 * c + j) * kVL], ps[j]);
        site[c] = cscale(t, csign);
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const C x = widen<C>(pin[c * kVL]);
      C q;
      if constexpr (CL) q = site[c];
      else q = cscale(x, diag);
#pragma unroll
      for (int src = 0; src < 4; ++src) {
        // the slot is read for every src (src == mu: slot 3 src, a valid one whose
        // value is not used) so that the choice below is between values: a choice
        // between the LDS slot and the wavefront's own partial as addresses put
        // the partial in private memory behind a generic load
        const C other = xch[3 * src + (mu < src ? mu : mu > src ? mu - 1 : 0)][c][lane];
        q = q + (src == mu ? (c == 0 ? m0 : c == 1 ? m1 : m2) : other);
      }
      if (live) {
        pout[c * kVL] = q;
        v0 += double(q.x) * x.x + double(q.y) * x.y;
        v1 += double(q.x) * x.y - double(q.y) * x.x;
        v2 += double(q.x) * q.x + double(q.y) * q.y;
      }
    }
    if (partial != nullptr) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        v0 += __shfl_xor(v0, o);
        v1 += __shfl_xor(v1, o);
        v2 += __shfl_xor(v2, o);
      }
      if (lane == 0) { red[mu][r][0] = v0; red[mu][r][1] = v1; red[mu][r][2] = v2; }
    }
    __syncthreads();  // the exchange slots are rewritten by the next RHS
  }
  if (partial == nullptr) return;
  for (int t = threadIdx.x; t < 3 * nrhs; t += blockDim.x) {
    const int r = t / 3, v = t % 3;
    partial[(blk * nrhs + r) * 3 + v] = red[0][r][v] + red[1][r][v] + red[2][r][v] + red[3][r][v];
  }
}

template <int FORM, int FIN = FORM>
void launch_wilson_dir(const WilsonArgs& a, hipStream_t st) {
  const int64_t nblk = (a.V + kVL - 1) / kVL;
  FineView<FIN> in(const_cast<void*>(a.in), a.V, a.nrhs);
  FineView<FORM> out(a.out, a.V, a.nrhs);
  GaugeView<FORM> U{static_cast<const typename Prec<FORM>::store*>(a.gauge), pad_sites(a.V)};
  const double4 hw = make_double4(a.hw[0], a.hw[1], a.hw[2], a.hw[3]);
  if (a.clover)
    hipLaunchKernelGGL((wilson_dir_kernel<FORM, FIN, true>), dim3(unsigned(nblk)), dim3(256), 0, st, in, out, U,
                       a.nbr, a.V, a.nrhs, typename Prec<FORM>::real(a.diag), hw, a.partial, a.swizzle, a.clover,
                       typename Prec<FORM>::real(a.clover_sign));
  else
    hipLaunchKernelGGL((wilson_dir_kernel<FORM, FIN, false>), dim3(unsigned(nblk)), dim3(256), 0, st, in, out, U,
                       a.nbr, a.V, a.nrhs, typename Prec<FORM>::real(a.diag), hw, a.partial, a.swizzle, a.clover,
                       typename Prec<FORM>::real(a.clover_sign));
  CRK_LAUNCH_CHECK();
}

template <int FORM, int R>
void launch_wilson(const WilsonArgs& a, hipStream_t st) {
  const int ngroups = (a.nrhs + R - 1) / R;
  const int64_t nsb = (a.V + 255) / 256;
  const int64_t nblk = nsb * ngroups;
  if (nblk > 0x7fffffff) fail(CRK_EINVAL, "dslash grid too large");
  FineView<FORM> in(const_cast<void*>(a.in), a.V, a.nrhs), out(a.out, a.V, a.nrhs);
  GaugeView<FORM> U{static_cast<const typename Prec<FORM>::store*>(a.gauge), pad_sites(a.V)};
  float4 hwf = make_float4(float(a.hw[0]), float(a.hw[1]), float(a.hw[2]), float(a.hw[3]));
  double4 hwd = make_double4(a.hw[0], a.hw[1], a.hw[2], a.hw[3]);
  if (a.clover)
    hipLaunchKernelGGL((wilson_kernel<FORM, R, true>), dim3(unsigned(nblk)), dim3(256), 0, st, in, out, U, a.nbr, a.V,
                       a.nrhs, ngroups, typename Prec<FORM>::real(a.diag), hwf, hwd, a.partial, nsb, a.order,
                       a.swizzle, a.clover, typename Prec<FORM>::real(a.clover_sign));
  else
    hipLaunchKernelGGL((wilson_kernel<FORM, R, false>), dim3(unsigned(nblk)), dim3(256), 0, st, in, out, U, a.nbr,
                       a.V, a.nrhs, ngroups, typename Prec<FORM>::real(a.diag), hwf, hwd, a.partial, nsb, a.order,
                       a.swizzle, a.clover, typename Prec<FORM>::real(a.clover_sign));
  CRK_LAUNCH_CHECK();
}


// ---------------------------------------------------------------- tile kernel
// Variant for the fine level of a hierarchy with 4^4 blocks (FP32, or FP16
// storage with FP32 arithmetic), whose device order is block-major: one
// workgroup owns one block (256 consecutive
// positions, one thread per site) and keeps the site's eight links in
// registers for the whole loop over right-hand sides.  Per RHS the workgroup
// stages the block's 256 spinors and the 512 spinors just outside its eight
// faces (64 per face) in LDS, then every hop reads its neighbour from LDS.
// Each spinor then passes through the vector cache three times per RHS (once
// as a block site, twice on average as a face neighbour) instead of nine, which
// is what bounds the one-thread-per-site kernels: their time follows the
// number of cache lines the neighbour gathers touch, not the bytes.  The block
// spinor of the next RHS is loaded while the current one is computed; the
// per-site arithmetic and its order are those of the other kernels.
constexpr int kTile = 256;                   // sites per block
constexpr int kTileSlots = kTile + 8 * 64;   // block sites, then face neighbours [dir][64]

// Index of block-local site l = l0 + 4 l1 + 16 l2 + 64 l3 on a face normal to mu:
// its local index with coordinate mu removed.
__device__ __forceinline__ int tile_face_index(int l, int mu) {
  const int lo = (1 << (2 * mu)) - 1;
  return (l & lo) | ((l >> (2 * mu + 2)) << (2 * mu));
}
// Inverse: the block-local site with face index i and coordinate mu = lmu.
__device__ __forceinline__ int tile_face_site(int i, int mu, int lmu) {
  const int lo = (1 << (2 * mu)) - 1;
  return (i & lo) | (lmu << (2 * mu)) | ((i >> (2 * mu)) << (2 * mu + 2));
}

// Links are held in their storage type (half2 links take half the registers)
// and widened per hop.
template <int MU, int SIGN, class S>
__device__ __forceinline__ void tile_hop(const float2 (*sp)[kTileSlots], int slot, const S (&us)[9],
                                         float2 (&acc)[12], float coef) {
  float2 psi[12], h[6], g[6], u[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    if constexpr (sizeof(S) == sizeof(float2)) {
      u[e] = us[e];
    } else {
      // widened here on every use: the empty asm keeps the compiler from
      // hoisting 144 widened registers out of the RHS loop
      uint32_t bits = __builtin_bit_cast(uint32_t, us[e]);
      asm volatile("" : "+v"(bits));
      u[e] = __half22float2(__builtin_bit_cast(__half2, bits));
    }
  }
#pragma unroll
  for (int c = 0; c < 12; ++c) psi[c] = sp[c][slot];
  project<MU, SIGN>(psi, h);
  link_mul<SIGN>(u, h, g);
  accumulate<MU, SIGN>(acc, g, coef);
}

// With the clover term the site blocks add to the live registers: that variant
// runs one workgroup per CU (up to 512 registers) instead of spilling.
template <int FORM, bool CL, bool SUB = false>  // FP32, or FP16S storage (half spinors with a per-site scale, half links) in FP32 arithmetic
__global__ __launch_bounds__(kTile, CL ? 1 : 2) void wilson_tile_kernel(FineView<FORM> in, FineView<FORM> out,
                                                               GaugeView<FORM> U,
                                                               const int* __restrict__ nbr, int64_t V, int nrhs,
                                                               float diag, float4 hw, double* __restrict__ partial,
                                                               int swz, const float2* __restrict__ clv, float csign,
                                                               const float2* __restrict__ sub) {
  __shared__ float2 sp[12][kTileSlots];  // [component][slot], 72 KiB
  const int64_t blk = swz ? xcd_swizzle(blockIdx.x, gridDim.x) : blockIdx.x;
  const int l = threadIdx.x, lane = l & 63, wid = l >> 6;
  const int64_t s = blk * kTile + l;
  // LDS slot of each neighbour, and the eight links
  int slot[8];
  typename Prec<FORM>::store u[8][9];
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    const int mu = d >> 1, lmu = (l >> (2 * mu)) & 3;
    const bool fwd = (d & 1) == 0;
    const bool inside = fwd ? lmu < 3 : lmu > 0;
    slot[d] = inside ? (fwd ? l + (1 << (2 * mu)) : l - (1 << (2 * mu))) : kTile + 64 * d + tile_face_index(l, mu);
    const int64_t y = fwd ? s : int64_t(nbr[int64_t(d) * V + s]);
    const typename Prec<FORM>::store* p = U.data + aidx(mu, 0, y, U.Vp, 9);
#pragma unroll
    for (int e = 0; e < 9; ++e) u[d][e] = p[e * kVL];
  }
  // the two face neighbours this thread stages: directions wid and 4 + wid, face index lane
  int64_t hy[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int d = 4 * k + wid, mu = d >> 1;
    hy[k] = nbr[int64_t(d) * V + blk * kTile + tile_face_site(lane, mu, (d & 1) ? 0 : 3)];
  }
  float2 own[12];
  in.load(0, s, own);
  for (int r = 0; r < nrhs; ++r) {
    {
      float2 f0[12], f1[12];
      in.load(r, hy[0], f0);
      in.load(r, hy[1], f1);
      __syncthreads();  // every thread is done with the previous RHS's tile
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        sp[c][l] = own[c];
        sp[c][kTile + l] = f0[c];
        sp[c][2 * kTile + l] = f1[c];
      }
      __syncthreads();
    }
    in.load(r + 1 < nrhs ? r + 1 : r, s, own);  // next RHS, in flight during the hops
    float2 acc[12];
    if constexpr (CL) {
      float2 ps[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) ps[c] = sp[c][l];
      clover_site(clv, in.Vp, s, ps, acc, csign);
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = cscale(sp[c][l], diag);
    }
    tile_hop<0, +1>(sp, slot[0], u[0], acc, hw.x);
    tile_hop<0, -1>(sp, slot[1], u[1], acc, hw.x);
    tile_hop<1, +1>(sp, slot[2], u[2], acc, hw.y);
    tile_hop<1, -1>(sp, slot[3], u[3], acc, hw.y);
    tile_hop<2, +1>(sp, slot[4], u[4], acc, hw.z);
    tile_hop<2, -1>(sp, slot[5], u[5], acc, hw.z);
    tile_hop<3, +1>(sp, slot[6], u[6], acc, hw.w);
    tile_hop<3, -1>(sp, slot[7], u[7], acc, hw.w);
    if constexpr (FORM == CRK_FORM_FP32) {
      // streaming stores: the output is not read again by this launch, so it
      // does not displace from L2 the spinors that neighbouring blocks still
      // read as face neighbours
      typedef float v2f __attribute__((ext_vector_type(2)));
      float2* po = out.data + aidx(r, 0, s, out.Vp, 12);
      // sub (FP32 only): out = sub - D in, the residual of the next step formed here
      const float2* pb = sub + aidx(r, 0, s, out.Vp, 12);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        v2f v;
        v.x = acc[c].x;
        v.y = acc[c].y;
        if constexpr (SUB) {
          const float2 b = pb[c * kVL];
          v.x = b.x - v.x;
          v.y = b.y - v.y;
        }
        __builtin_nontemporal_store(v, reinterpret_cast<v2f*>(po + c * kVL));
      }
    } else {
      out.store(r, s, acc);  // rescaled to the site's largest component
    }
    if (partial != nullptr) {
      // the site's twelve terms in FP32 (the form's accumulation precision),
      // the sums over sites in FP64
      float f0 = 0, f1 = 0, f2 = 0;
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const float2 q = acc[c], x = sp[c][l];
        f0 += q.x * x.x + q.y * x.y;
        f1 += q.x * x.y - q.y * x.x;
        f2 += q.x * q.x + q.y * q.y;
      }
      double v0 = f0, v1 = f1, v2 = f2;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        v0 += __shfl_xor(v0, o);
        v1 += __shfl_xor(v1, o);
        v2 += __shfl_xor(v2, o);
      }
      // one partial row per wavefront (64 sites), as in the other kernels
      if (lane == 0) {
        double* p = partial + ((blk * 4 + wid) * nrhs + r) * 3;
        p[0] = v0;
        p[1] = v1;
        p[2] = v2;
      }
    }
  }
}

template <int FORM>
void launch_wilson_tile(const WilsonArgs& a, hipStream_t st) {
  CRK_REQUIRE(a.V % kTile == 0, "tile dslash: the volume must be a multiple of 4^4");
  const int64_t nblk = a.V / kTile;
  if (nblk > 0x7fffffff) fail(CRK_EINVAL, "dslash grid too large");
  FineView<FORM> in(const_cast<void*>(a.in), a.V, a.nrhs), out(a.out, a.V, a.nrhs);
  GaugeView<FORM> U{static_cast<const typename Prec<FORM>::store*>(a.gauge), pad_sites(a.V)};
  const float4 hw = make_float4(float(a.hw[0]), float(a.hw[1]), float(a.hw[2]), float(a.hw[3]));
  CRK_REQUIRE(a.sub == nullptr || (FORM == CRK_FORM_FP32 && a.partial == nullptr && a.clover == nullptr),
              "tile dslash: b - D x only in FP32, without fused sums or the clover term");
  const float2* sub = static_cast<const float2*>(a.sub);
  if (a.clover)
    hipLaunchKernelGGL((wilson_tile_kernel<FORM, true>), dim3(unsigned(nblk)), dim3(kTile), 0, st, in, out, U, a.nbr,
                       a.V, a.nrhs, float(a.diag), hw, a.partial, a.swizzle, static_cast<const float2*>(a.clover),
                       float(a.clover_sign), sub);
  else if (sub)
    hipLaunchKernelGGL((wilson_tile_kernel<FORM, false, FORM == CRK_FORM_FP32>), dim3(unsigned(nblk)), dim3(kTile), 0,
                       st, in, out, U, a.nbr, a.V, a.nrhs, float(a.diag), hw, a.partial, a.swizzle,
                       static_cast<const float2*>(a.clover), float(a.clover_sign), sub);
  else
    hipLaunchKernelGGL((wilson_tile_kernel<FORM, false>), dim3(unsigned(nblk)), dim3(kTile), 0, st, in, out, U, a.nbr,
                       a.V, a.nrhs, float(a.diag), hw, a.partial, a.swizzle, static_cast<const float2*>(a.clover),
                       float(a.clover_sign), sub);
  CRK_LAUNCH_CHECK();
}
}  // namespace

int64_t wilson_partial_blocks(int64_t V) { return (V + kVL - 1) / kVL; }

void wilson_apply(const WilsonArgs& a_in, hipStream_t st) {
  if (a_in.nrhs <= 0 || a_in.V <= 0) return;
  CRK_REQUIRE(a_in.in != a_in.out, "dslash: in and out must not alias");
  const WilsonArgs& a = a_in;
  if (a.in_form >= 0 && a.in_form != a.form) {
    // FP64 operator on FP32-stored input, in launches of at most kDirMaxRhs RHS
    CRK_REQUIRE(a.form == CRK_FORM_FP64 && a.in_form == CRK_FORM_FP32,
                "dslash: mixed storage only as FP32 input to the FP64 operator");
    CRK_REQUIRE(a.partial == nullptr || a.nrhs <= kDirMaxRhs, "dslash: fused sums need one launch");
    const int64_t per = 12 * pad_sites(a.V);
    for (int r0 = 0; r0 < a.nrhs; r0 += kDirMaxRhs) {
      WilsonArgs b = a;
      b.nrhs = a.nrhs - r0 < kDirMaxRhs ? a.nrhs - r0 : kDirMaxRhs;
      b.in = static_cast<const float2*>(a.in) + per * r0;
      b.out = static_cast<double2*>(a.out) + per * r0;
      launch_wilson_dir<CRK_FORM_FP64, CRK_FORM_FP32>(b, st);
    }
    return;
  }
  const int R = a.rhs_per_thread < a.nrhs ? a.rhs_per_thread : a.nrhs;
  CRK_REQUIRE(a.sub == nullptr || (a.tile4 && a.form == CRK_FORM_FP32), "dslash: b - D x only with the FP32 tile");
  if (a.tile4 && a.form == CRK_FORM_FP32) { launch_wilson_tile<CRK_FORM_FP32>(a, st); return; }
  if (a.tile4 && a.form == CRK_FORM_FP16S) { launch_wilson_tile<CRK_FORM_FP16S>(a, st); return; }
  if (a.form == CRK_FORM_FP32) { launch_wilson_rhsloop<CRK_FORM_FP32>(a, st); return; }
  if (a.nrhs <= kDirMaxRhs && a.form == CRK_FORM_FP64) { launch_wilson_dir<CRK_FORM_FP64>(a, st); return; }
  switch (a.form) {
    case CRK_FORM_FP64:
      if (R >= 4) launch_wilson<CRK_FORM_FP64, 4>(a, st);
      else if (R >= 2) launch_wilson<CRK_FORM_FP64, 2>(a, st);
      else launch_wilson<CRK_FORM_FP64, 1>(a, st);
      break;
    case CRK_FORM_FP32:
      if (R >= 8) launch_wilson<CRK_FORM_FP32, 8>(a, st);
      else if (R >= 4) launch_wilson<CRK_FORM_FP32, 4>(a, st);
      else if (R >= 2) launch_wilson<CRK_FORM_FP32, 2>(a, st);
      else launch_wilson<CRK_FORM_FP32, 1>(a, st);
      break;
    case CRK_FORM_FP16S:
      if (R >= 8) launch_wilson<CRK_FORM_FP16S, 8>(a, st);
      else if (R >= 4) launch_wilson<CRK_FORM_FP16S, 4>(a, st);
      else if (R >= 2) launch_wilson<CRK_FORM_FP16S, 2>(a, st);
      else launch_wilson<CRK_FORM_FP16S, 1>(a, st);
      break;
    default:
      fail(CRK_EINVAL, "unknown precision form");
  }
}

}  // namespace crk
