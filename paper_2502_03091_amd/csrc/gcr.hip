// Multi-RHS kernels of the flexible GCR solver (paper, Sec. 2 last paragraph:
// the hierarchy preconditions a flexible outer solver such as GCR).
//
// Every right-hand side runs its own GCR recursion; the kernels carry one set
// of scalars per RHS and a per-RHS active flag, so RHS that have converged are
// frozen without a host round trip.  Per iteration (slot i):
//   c_j   = <w_j, w_i>           for the valid stored directions j     (multidot)
//   w_i  -= sum_j c_j w_j ; z_i -= sum_j c_j z_j   (classical Gram-Schmidt)
//   a     = <w_i, r>/||w_i|| ;  w_i, z_i /= ||w_i||
//   x    += a z_i ;  r -= a w_i ;  ||r||^2                          (update)
// The solvers use a lazy form of the same recursion: z_i is neither
// orthogonalised nor normalised and x is not updated per iteration; c_ij,
// 1/||w_i|| and a_i are recorded and the solution is formed from the raw z_i
// when it is needed, which saves the z and x traffic: once at the end of an
// inner solve (lazy_coef_kernel, lazy_solution_kernel), and for an outer slot
// over its window of the direction ring when it claims convergence, restarts
// or stops (ring_lazy_coef_kernel, ring_lazy_x_kernel).
// Reductions are deterministic (fixed thread ranges, fixed trees, fixed-order
// final sums).  Fields are addressed as entry e of rhs r at r*rs + e*es.
#include "gcr.h"

#include <algorithm>

namespace crk {

namespace {

constexpr int kT = 256;
// Loads in flight per thread in the single-workgroup reductions (multidot
// coefficients, convergence check): a few hundred rows per wavefront are
// latency-bound, not bandwidth-bound.
constexpr int kRedLoads = 32;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

int64_t chunk_of(int64_t n) {
  int64_t c = (n + 511) / 512;
  return c < 2048 ? 2048 : c;
}

// Elements per workgroup chunk: rhs-outer fields use long chunks (coalesced
// runs of one RHS); rhs-inner fields use one element per thread so that the
// small coarse fields still spread over many workgroups.  Either way the chunk
// depends on n only, so an RHS's sums do not depend on the number of RHS.
int64_t chunk_for_shape(int64_t n, bool inner) { return inner ? int64_t(kInnerChunk) : chunk_of(n); }

// Directions per multidot workgroup: grid z runs over groups of kDotGroup
// stored directions, so a thread keeps 2*kDotGroup sums and issues the loads
// of all its group's directions together.  The last group repeats the last
// direction for its unused members (in-bounds loads, sums not stored).
constexpr int kDotGroup = 16;

// partial[chunk][r][2*j + {0,1}] = chunk sum of conj(W_j) w.  G directions per
// workgroup (4, 8 or 16, the smallest that holds the pass): fewer unused sums
// keep fewer registers live and more wavefronts in flight; an entry's sum does
// not depend on G.  valid (optional): bit vbit0 + j of valid[r] set when
// direction j belongs to RHS r's basis; the others are neither read nor summed
// (their partials are 0, and their coefficients are zeroed when reduced).
template <class C, int G>
__global__ __launch_bounds__(kT) void multidot_kernel(const C* __restrict__ Wb, int64_t fstride, int nj,
                                                      const C* __restrict__ w, int64_t n, int nrhs, int64_t rs,
                                                      int64_t es, int64_t chunk, double* __restrict__ partial,
                                                      const uint32_t* __restrict__ valid, int vbit0) {
  __shared__ double sh[2 * G][4];
  const int r = blockIdx.y, j0 = blockIdx.z * G;
  const int64_t e0 = int64_t(blockIdx.x) * chunk, e1 = min(n, e0 + chunk);
  const C* Wg[G];
#pragma unroll
  for (int g = 0; g < G; ++g) Wg[g] = Wb + int64_t(min(j0 + g, nj - 1)) * fstride;
  double acc[2 * G];
#pragma unroll
  for (int q = 0; q < 2 * G; ++q) acc[q] = 0;
  // members past the group's last direction, and directions outside this
  // RHS's basis, issue no loads (both are uniform over the workgroup, whose RHS
  // is blockIdx.y, so the branches are too)
  const int ng = min(G, nj - j0);
  const uint32_t vm = valid ? valid[r] >> (vbit0 + j0) : ~0u;
  bool use[G];
#pragma unroll
  for (int g = 0; g < G; ++g) use[g] = g < ng && ((vm >> g) & 1u);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int64_t idx = int64_t(r) * rs + e * es;
    const C y = w[idx];
    C x[G];
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (use[g]) x[g] = Wg[g][idx];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (use[g]) {
        acc[2 * g] += double(x[g].x) * y.x + double(x[g].y) * y.y;
        acc[2 * g + 1] += double(x[g].x) * y.y - double(x[g].y) * y.x;
      }
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 2 * G; ++q) {
    const double t = wsum(acc[q]);
    if (lane == 0) sh[q][wid] = t;
  }
  __syncthreads();
  const int nq = 2 * min(G, nj - j0);
  for (int q = threadIdx.x; q < nq; q += blockDim.x)
    partial[(int64_t(blockIdx.x) * nrhs + r) * (2 * kMaxBasis) + 2 * j0 + q] =
        sh[q][0] + sh[q][1] + sh[q][2] + sh[q][3];
}

// Rhs-inner fields: one wavefront per (chunk of kInnerChunk elements, rhs);
// lane l sums elements l, l + 64, ... of the chunk in order, then the lanes'
// sums are transposed through LDS and lane q adds value q of lanes 0..63 in
// order (64 LDS reads instead of a shuffle tree per value).
template <class C>
__global__ __launch_bounds__(64) void multidot_inner_kernel(const C* __restrict__ Wb, int64_t fstride, int nj,
                                                            const C* __restrict__ w, int64_t n, int nrhs,
                                                            int64_t rs, int64_t es, double* __restrict__ partial) {
  __shared__ double sh[64][2 * kDotGroup + 1];
  const int r = blockIdx.y, l = threadIdx.x, j0 = blockIdx.z * kDotGroup;
  const int64_t c = blockIdx.x;
  const C* Wg[kDotGroup];
#pragma unroll
  for (int g = 0; g < kDotGroup; ++g) Wg[g] = Wb + int64_t(min(j0 + g, nj - 1)) * fstride;
  double acc[2 * kDotGroup];
#pragma unroll
  for (int q = 0; q < 2 * kDotGroup; ++q) acc[q] = 0;
  for (int i = 0; i < kInnerChunk / 64; ++i) {
    const int64_t e = c * kInnerChunk + l + 64 * i;
    if (e >= n) break;
    const int64_t idx = int64_t(r) * rs + e * es;
    const C y = w[idx];
    C x[kDotGroup];
#pragma unroll
    for (int g = 0; g < kDotGroup; ++g) x[g] = Wg[g][idx];
#pragma unroll
    for (int g = 0; g < kDotGroup; ++g) {
      acc[2 * g] += double(x[g].x) * y.x + double(x[g].y) * y.y;
      acc[2 * g + 1] += double(x[g].x) * y.y - double(x[g].y) * y.x;
    }
  }
#pragma unroll
  for (int q = 0; q < 2 * kDotGroup; ++q) sh[l][q] = acc[q];
  __syncthreads();
  if (l < 2 * min(kDotGroup, nj - j0)) {
    double t = 0;
    for (int k = 0; k < 64; ++k) t += sh[k][l];
    partial[(c * nrhs + r) * (2 * kMaxBasis) + 2 * j0 + l] = t;
  }
}

// Same sums for rhs-inner fields with a workgroup per (chunk, group of up to
// 16 RHS, group of kInnerGroup directions): thread (l, r) with r fastest, so a
// wavefront reads contiguous RHS runs of consecutive entries.  Each (l, r)
// thread adds entries l, l + 64, ... of the chunk in order and the 64 lane
// sums of an RHS are added in lane order, exactly as in multidot_inner_kernel,
// so the partials are the same numbers.
constexpr int kInnerGroup = 4;
constexpr int kInnerRhs = 16;

template <class C>
__global__ __launch_bounds__(64 * kInnerRhs) void multidot_inner_rg_kernel(const C* __restrict__ Wb, int64_t fstride,
                                                                           int nj, const C* __restrict__ w, int64_t n,
                                                                           int nrhs, double* __restrict__ partial) {
  __shared__ double sh[64][kInnerRhs][2 * kInnerGroup + 1];  // [lane][rhs]: the RHS of a lane in different banks
  const int rg = min(kInnerRhs, nrhs - int(blockIdx.y) * kInnerRhs);  // RHS in this workgroup
  const int t = threadIdx.x;
  const int rl = t % rg, l = t / rg;
  const int r = int(blockIdx.y) * kInnerRhs + rl;
  const int j0 = blockIdx.z * kInnerGroup;
  const int64_t c = blockIdx.x;
  const C* Wg[kInnerGroup];
#pragma unroll
  for (int g = 0; g < kInnerGroup; ++g) Wg[g] = Wb + int64_t(min(j0 + g, nj - 1)) * fstride;
  if (l < 64) {
    double acc[2 * kInnerGroup];
#pragma unroll
    for (int q = 0; q < 2 * kInnerGroup; ++q) acc[q] = 0;
    for (int i = 0; i < kInnerChunk / 64; ++i) {
      const int64_t e = c * kInnerChunk + l + 64 * i;
      if (e >= n) break;
      const int64_t idx = e * nrhs + r;
      const C y = w[idx];
      C x[kInnerGroup];
#pragma unroll
      for (int g = 0; g < kInnerGroup; ++g) x[g] = Wg[g][idx];
#pragma unroll
      for (int g = 0; g < kInnerGroup; ++g) {
        acc[2 * g] += double(x[g].x) * y.x + double(x[g].y) * y.y;
        acc[2 * g + 1] += double(x[g].x) * y.y - double(x[g].y) * y.x;
      }
    }
#pragma unroll
    for (int q = 0; q < 2 * kInnerGroup; ++q) sh[l][rl][q] = acc[q];
  }
  __syncthreads();
  const int nq = 2 * min(kInnerGroup, nj - j0);
  if (t < rg * nq) {
    const int rr = t / nq, q = t % nq;
    double s = 0;
    for (int k = 0; k < 64; ++k) s += sh[k][rr][q];
    partial[(c * nrhs + int(blockIdx.y) * kInnerRhs + rr) * (2 * kMaxBasis) + 2 * j0 + q] = s;
  }
}

// coef[r][j0 + j] = valid(r, j0 + j) ? sum over chunks : 0.  One workgroup per
// rhs; wavefront g sums chunks g, g + 4, ... in order for every value q (lane q),
// then the four wavefront sums are added in a fixed order.
__global__ __launch_bounds__(kT) void multidot_reduce_kernel(const double* __restrict__ partial, int64_t nch, int nrhs,
                                                             int j0, int nj, const uint32_t* __restrict__ valid,
                                                             double2* __restrict__ coef) {
  __shared__ double sh[kT / 64][2 * kMaxBasis];
  const int r = blockIdx.x;
  const int q = threadIdx.x & 63, g = threadIdx.x >> 6;
  double acc = 0;
  if (q < 2 * nj) {
    // loads issued kRedLoads at a time (the kernel is bound by their latency),
    // added in chunk order
    for (int64_t c0 = g; c0 < nch; c0 += kRedLoads * (kT / 64)) {
      double v[kRedLoads];
#pragma unroll
      for (int u = 0; u < kRedLoads; ++u) {
        const int64_t c = c0 + int64_t(u) * (kT / 64);
        v[u] = c < nch ? partial[(c * nrhs + r) * (2 * kMaxBasis) + q] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kRedLoads; ++u)
        if (c0 + int64_t(u) * (kT / 64) < nch) acc += v[u];
    }
  }
  sh[g][q] = acc;
  __syncthreads();
  for (int j = threadIdx.x; j < nj; j += blockDim.x) {
    const double re = ((sh[0][2 * j] + sh[1][2 * j]) + sh[2][2 * j]) + sh[3][2 * j];
    const double im = ((sh[0][2 * j + 1] + sh[1][2 * j + 1]) + sh[2][2 * j + 1]) + sh[3][2 * j + 1];
    const bool ok = valid ? ((valid[r] >> (j0 + j)) & 1u) : true;
    coef[r * kMaxCoef + j0 + j] = ok ? make_double2(re, im) : make_double2(0, 0);
  }
}

// w -= sum_j coef_j W_j, summed from stored slot j_first
// onwards (cyclically), i.e. oldest direction first: the rounding of an RHS's
// update then depends only on its own directions, not on where in a ring they sit.
template <class C>
__global__ __launch_bounds__(kT) void multiaxpy_kernel(const C* __restrict__ Wb, int64_t fstride, int nj, int j_first,
                                                       C* __restrict__ w, const double2* __restrict__ coef, int64_t n,
                                                       int nrhs, int64_t rs, int64_t es) {
  constexpr int kU = 4;  // directions whose loads are issued together
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * nrhs) return;
  const int r = es == 1 ? int(t / n) : int(t % nrhs);
  const int64_t e = es == 1 ? t % n : t / nrhs;
  const int64_t idx = int64_t(r) * rs + e * es;
  using T = decltype(C::x);
  C ww = w[idx];
  for (int t0 = 0; t0 < nj; t0 += kU) {
    C wl[kU], c[kU];
    int jj[kU];
    bool on[kU];
    // coefficients first, so that the direction loads below are issued back to back
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      // past the end: the last direction's index (in bounds), skipped
      const int tt = t0 + u < nj ? t0 + u : nj - 1;
      jj[u] = tt + j_first < nj ? tt + j_first : tt + j_first - nj;
      const double2 cd = coef[r * kMaxCoef + jj[u]];
      on[u] = t0 + u < nj && (cd.x != 0.0 || cd.y != 0.0);  // zero: an unused slot or a frozen RHS, not read
      c[u] = mk<C>(T(-cd.x), T(-cd.y));
    }
    // nothing to add (unused slots, or a frozen RHS): no loads at all
    bool any = false;
#pragma unroll
    for (int u = 0; u < kU; ++u) any |= on[u];
    if (!any) continue;
    // a skipped direction re-reads this thread's own w entry (already in
    // cache) instead of branching, so all loads stay in flight together
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t off = on[u] ? jj[u] * fstride + idx : idx;
      wl[u] = (on[u] ? Wb : static_cast<const C*>(w))[off];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (on[u]) cfma(ww, c[u], wl[u]);
    }
  }
  w[idx] = ww;
}

// update with the scalars computed in place: every workgroup of RHS r first adds
// the <w, r>, ||w||^2 partials of its RHS (lane l takes chunks l, l + 64, ... in
// order, then a fixed shuffle tree; the same in every workgroup) and derives
// inv = 1/||w|| and a = <w, r>/||w||, which saves the reduction and scalar launches.
// Then w *= inv and r -= a w; inv and a go to hinv[r], ha[r] (the solution is
// formed later from the recorded recursion), and ||r||^2 to the partials.
template <class C>
__global__ __launch_bounds__(kT) void update_fused_kernel(C* __restrict__ w, C* __restrict__ res,
                                                          const double* __restrict__ dpart,
                                                          int64_t dnch, const int* __restrict__ active,
                                                          int* __restrict__ breakdown, int64_t n, int nrhs,
                                                          int64_t rs, int64_t es, int64_t chunk,
                                                          double* __restrict__ partial, double* __restrict__ hinv,
                                                          double2* __restrict__ ha) {
  __shared__ double sh[4];
  __shared__ double scal[3];
  using T = decltype(C::x);
  const int r = blockIdx.y;
  if (threadIdx.x < 64) {
    double s0 = 0, s1 = 0, s2 = 0;
    for (int64_t c = threadIdx.x; c < dnch; c += 64) {
      const double* p = dpart + (c * nrhs + r) * 3;
      s0 += p[0];
      s1 += p[1];
      s2 += p[2];
    }
    s0 = wsum(s0);
    s1 = wsum(s1);
    s2 = wsum(s2);
    if (threadIdx.x == 0) {
      scal[0] = s0;
      scal[1] = s1;
      scal[2] = s2;
    }
  }
  __syncthreads();
  const double ww = scal[2], nw = sqrt(ww);
  const bool act0 = active[r] != 0;
  const bool ok = act0 && ww > 0.0 && isfinite(nw);
  if (blockIdx.x == 0 && threadIdx.x == 0 && breakdown) breakdown[r] = act0 && !ok;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    hinv[r] = ok ? 1.0 / nw : 0.0;
    ha[r] = ok ? make_double2(scal[0] / nw, scal[1] / nw) : make_double2(0, 0);
  }
  const T s = T(ok ? 1.0 / nw : 0.0);
  const bool act = ok;
  const C ar = ok ? mk<C>(T(scal[0] / nw), T(scal[1] / nw)) : mk<C>(T(0), T(0));
  const int64_t e0 = int64_t(blockIdx.x) * chunk, e1 = min(n, e0 + chunk);
  double acc = 0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int64_t idx = int64_t(r) * rs + e * es;
    const C wn = cscale(w[idx], s);
    w[idx] = wn;
    C rr = res[idx];
    if (act) {
      const C aw = cmul(ar, wn);
      rr.x -= aw.x;
      rr.y -= aw.y;
      res[idx] = rr;
    }
    acc += double(rr.x) * rr.x + double(rr.y) * rr.y;
  }
  const double t = wsum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) partial[int64_t(blockIdx.x) * nrhs + r] = sh[0] + sh[1] + sh[2] + sh[3];
}

// One-pass step of the outer solve on rhs-outer fields whose stored
// directions sit in a ring (the formulas of gs_update_rg_kernel below):
// ||w^||^2 = ||w||^2 - sum_j |c_j|^2 and <w^, r> = <w, r> from the multidot
// coefficients and the dots of the unmodified w, then one pass forms
// w^ = w - sum_j c_j W_j (the ring from slot j_first on, oldest first; slots
// with a zero coefficient, outside the RHS's basis, are not read: the same
// sum, in the same order, as multiaxpy_kernel), stores w^/||w^|| and updates
// r -= a w^/||w^|| with the ||r||^2 partials.  Workgroup per (chunk, RHS):
// every workgroup of RHS r adds the dot partials and the coefficients of its
// RHS in the same order, so all of them use the same scalars.
template <class C>
__global__ __launch_bounds__(kT) void gs_update_ring_kernel(
    const C* __restrict__ Wb, int64_t fstride, int nj, int j_first, C* __restrict__ w, C* __restrict__ res,
    const double2* __restrict__ coef, const double* __restrict__ dpart, int64_t dnch, const int* __restrict__ active,
    int* __restrict__ breakdown, int64_t n, int nrhs, int64_t rs, int64_t chunk, double* __restrict__ partial,
    double* __restrict__ hinv, double2* __restrict__ ha, double rel) {
  __shared__ double sh[4];
  __shared__ double scal[3];
  __shared__ double2 cf[kMaxCoef];
  __shared__ int slot[kMaxCoef];
  __shared__ int nuse;
  using T = decltype(C::x);
  const int r = blockIdx.y;
  if (threadIdx.x < 64) {
    double s0 = 0, s1 = 0, s2 = 0;
    for (int64_t c = threadIdx.x; c < dnch; c += 64) {
      const double* p = dpart + (c * nrhs + r) * 3;
      s0 += p[0];
      s1 += p[1];
      s2 += p[2];
    }
    s0 = wsum(s0);
    s1 = wsum(s1);
    s2 = wsum(s2);
    if (threadIdx.x == 0) {
      scal[0] = s0;
      scal[1] = s1;
      scal[2] = s2;
      int m = 0;
      for (int tt = 0; tt < nj; ++tt) {
        const int j = tt + j_first < nj ? tt + j_first : tt + j_first - nj;
        const double2 cd = coef[r * kMaxCoef + j];
        if (cd.x != 0.0 || cd.y != 0.0) {
          cf[m] = cd;
          slot[m] = j;
          ++m;
        }
      }
      nuse = m;
    }
  }
  __syncthreads();
  const int m = nuse;
  double c2 = 0;
  for (int u = 0; u < m; ++u) c2 += cf[u].x * cf[u].x + cf[u].y * cf[u].y;
  const double s2 = scal[2], hw2 = s2 - c2;
  const bool act0 = active[r] != 0;
  const bool ok = act0 && s2 > 0.0 && hw2 > rel * s2 && isfinite(hw2);
  const double nw = sqrt(hw2), inv = ok ? 1.0 / nw : 0.0;
  const double2 a = ok ? make_double2(scal[0] / nw, scal[1] / nw) : make_double2(0, 0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (breakdown) breakdown[r] = act0 && !ok;
    hinv[r] = inv;
    ha[r] = a;
  }
  const T s = T(inv);
  const C ar = mk<C>(T(a.x), T(a.y));
  const int64_t e0 = int64_t(blockIdx.x) * chunk, e1 = min(n, e0 + chunk);
  double racc = 0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int64_t idx = int64_t(r) * rs + e;
    C ww = w[idx];
    if (ok) {
      constexpr int kU = 4;  // directions whose loads are issued together
      for (int u0 = 0; u0 < m; u0 += kU) {
        C wl[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) wl[u] = Wb[int64_t(slot[min(u0 + u, m - 1)]) * fstride + idx];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          if (u0 + u < m) {
            const C c = mk<C>(T(-cf[u0 + u].x), T(-cf[u0 + u].y));
            cfma(ww, c, wl[u]);
          }
        }
      }
    }
    const C wn = cscale(ww, s);
    w[idx] = wn;
    C rr = res[idx];
    if (ok) {
      const C aw = cmul(ar, wn);
      rr.x -= aw.x;
      rr.y -= aw.y;
      res[idx] = rr;
    }
    racc += double(rr.x) * rr.x + double(rr.y) * rr.y;
  }
  const double t = wsum(racc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) partial[int64_t(blockIdx.x) * nrhs + r] = sh[0] + sh[1] + sh[2] + sh[3];
}

// update_fused_kernel for rhs-inner fields: workgroup per (chunk, group of up
// to 16 RHS), thread (l, r) with r fastest (coalesced), entries l, l + 64, ...
// of the chunk per thread; every sum over lanes runs in lane order, so an RHS's
// numbers do not depend on how many RHS share the field.
template <class C>
__global__ __launch_bounds__(64 * kInnerRhs) void update_fused_rg_kernel(C* __restrict__ w, C* __restrict__ res,
                                                                         const double* __restrict__ dpart,
                                                                         int64_t dnch, const int* __restrict__ active,
                                                                         int* __restrict__ breakdown, int64_t n,
                                                                         int nrhs, double* __restrict__ partial,
                                                                         double* __restrict__ hinv,
                                                                         double2* __restrict__ ha) {
  __shared__ double sh[64][kInnerRhs][3];  // [lane][rhs]: the RHS of a lane in different banks
  __shared__ double scal[kInnerRhs][3];
  using T = decltype(C::x);
  const int rg = min(kInnerRhs, nrhs - int(blockIdx.y) * kInnerRhs);
  const int t = threadIdx.x;
  const int rl = t % rg, l = t / rg;
  const int r = int(blockIdx.y) * kInnerRhs + rl;
  // (<w, r>, ||w||^2) of each RHS from the dot partials
  if (l < 64) {
    double s0 = 0, s1 = 0, s2 = 0;
    for (int64_t c = l; c < dnch; c += 64) {
      const double* p = dpart + (c * nrhs + r) * 3;
      s0 += p[0];
      s1 += p[1];
      s2 += p[2];
    }
    sh[l][rl][0] = s0;
    sh[l][rl][1] = s1;
    sh[l][rl][2] = s2;
  }
  __syncthreads();
  if (t < 3 * rg) {
    const int rr = t / 3, v = t % 3;
    double a = 0;
    for (int k = 0; k < 64; ++k) a += sh[k][rr][v];
    scal[rr][v] = a;
  }
  __syncthreads();
  double acc = 0;
  if (l < 64) {
    const double ww = scal[rl][2], nw = sqrt(ww);
    const bool act0 = active[r] != 0;
    const bool ok = act0 && ww > 0.0 && isfinite(nw);
    if (blockIdx.x == 0 && l == 0 && breakdown) breakdown[r] = act0 && !ok;
    if (blockIdx.x == 0 && l == 0) {
      hinv[r] = ok ? 1.0 / nw : 0.0;
      ha[r] = ok ? make_double2(scal[rl][0] / nw, scal[rl][1] / nw) : make_double2(0, 0);
    }
    const T sc = T(ok ? 1.0 / nw : 0.0);
    const C ar = ok ? mk<C>(T(scal[rl][0] / nw), T(scal[rl][1] / nw)) : mk<C>(T(0), T(0));
    for (int i = 0; i < kInnerChunk / 64; ++i) {
      const int64_t e = int64_t(blockIdx.x) * kInnerChunk + l + 64 * i;
      if (e >= n) break;
      const int64_t idx = e * nrhs + r;
      const C wn = cscale(w[idx], sc);
      w[idx] = wn;
      C rr = res[idx];
      if (ok) {
        const C aw = cmul(ar, wn);
        rr.x -= aw.x;
        rr.y -= aw.y;
        res[idx] = rr;
      }
      acc += double(rr.x) * rr.x + double(rr.y) * rr.y;
    }
  }
  __syncthreads();  // sh is reused
  if (l < 64) sh[l][rl][0] = acc;
  __syncthreads();
  if (t < rg) {
    double a = 0;
    for (int k = 0; k < 64; ++k) a += sh[k][t][0];
    partial[int64_t(blockIdx.x) * nrhs + int(blockIdx.y) * kInnerRhs + t] = a;
  }
}

// One-pass step of an inner solve on rhs-inner (coarse) fields.  With the
// Gram-Schmidt coefficients c_j = <W_j, w> of the stored orthonormal
// directions (multidot) and the dots of the unmodified w (rhs_dot partials:
// <w, r>, ||w||^2), the scalars of the step need no pass over the
// orthogonalised direction w^ = w - sum_j c_j W_j:
//   ||w^||^2 = ||w||^2 - sum_j |c_j|^2   (the W_j are orthonormal),
//   <w^, r>  = <w, r>                    (r is orthogonal to every stored W_j),
// so one pass forms w^, stores w^/||w^|| in place and updates
// r -= (<w^, r>/||w^||) w^/||w^||, with the ||r||^2 partials of the check.
// The recursion stays consistent whatever the rounding of these scalars:
// the stored direction is exactly A p_i of the recorded p_i, and r is updated
// with it.  A direction whose ||w^||^2 is not well above the rounding of
// ||w||^2 (w nearly in the span of the stored directions; rel is the relative
// floor for the vector precision) is a breakdown: the RHS's inner solve stops,
// as for a zero direction.  Workgroup per (chunk, group of up to 16 RHS),
// thread (l, r) with r fastest; the sums over lanes and chunks run in fixed
// orders, so an RHS's numbers do not depend on the other RHS of the field.
template <class C>
__global__ __launch_bounds__(64 * kInnerRhs) void gs_update_rg_kernel(
    const C* __restrict__ Wb, int64_t fstride, int nj, C* __restrict__ w, C* __restrict__ res,
    const double2* __restrict__ coef, const double* __restrict__ dpart, int64_t dnch, const int* __restrict__ active,
    int* __restrict__ breakdown, int64_t n, int nrhs, double* __restrict__ partial, double* __restrict__ hinv,
    double2* __restrict__ ha, double rel) {
  __shared__ double sh[64][kInnerRhs][3];  // [lane][rhs]: the RHS of a lane in different banks
  __shared__ double scal[kInnerRhs][3];  // 1/||w^||, Re a, Im a
  __shared__ double2 cf[kInnerRhs][kMaxCoef];
  using T = decltype(C::x);
  constexpr int kE = kInnerChunk / 64;  // entries per thread
  const int r0 = int(blockIdx.y) * kInnerRhs;
  const int rg = min(kInnerRhs, nrhs - r0);
  const int t = threadIdx.x;
  const int rl = t % rg, l = t / rg;
  const int r = r0 + rl;
  if (l < 64) {
    double s0 = 0, s1 = 0, s2 = 0;
    for (int64_t c = l; c < dnch; c += 64) {
      const double* p = dpart + (c * nrhs + r) * 3;
      s0 += p[0];
      s1 += p[1];
      s2 += p[2];
    }
    sh[l][rl][0] = s0;
    sh[l][rl][1] = s1;
    sh[l][rl][2] = s2;
  }
  for (int q = t; q < rg * nj; q += blockDim.x) cf[q / nj][q % nj] = coef[(r0 + q / nj) * kMaxCoef + q % nj];
  __syncthreads();
  if (t < 3 * rg) {
    const int rr = t / 3, v = t % 3;
    double a = 0;
    for (int k = 0; k < 64; ++k) a += sh[k][rr][v];
    scal[rr][v] = a;
  }
  __syncthreads();
  if (t < rg) {
    const double s0 = scal[t][0], s1 = scal[t][1], s2 = scal[t][2];
    double c2 = 0;
    for (int j = 0; j < nj; ++j) c2 += cf[t][j].x * cf[t][j].x + cf[t][j].y * cf[t][j].y;
    const double hw2 = s2 - c2;
    const bool act0 = active[r0 + t] != 0;
    const bool ok = act0 && s2 > 0.0 && hw2 > rel * s2 && isfinite(hw2);
    const double inv = ok ? 1.0 / sqrt(hw2) : 0.0;
    scal[t][0] = inv;
    scal[t][1] = s0 * inv;
    scal[t][2] = s1 * inv;
    if (blockIdx.x == 0) {
      if (breakdown) breakdown[r0 + t] = act0 && !ok;
      hinv[r0 + t] = inv;
      ha[r0 + t] = make_double2(s0 * inv, s1 * inv);
    }
  }
  __syncthreads();
  double racc = 0;
  if (l < 64) {
    const double inv = scal[rl][0];
    const bool ok = inv != 0.0;
    const C ar = mk<C>(T(scal[rl][1]), T(scal[rl][2]));
    int64_t idx[kE];
    bool in[kE];
    C acc[kE];
#pragma unroll
    for (int i = 0; i < kE; ++i) {
      const int64_t e = int64_t(blockIdx.x) * kInnerChunk + l + 64 * i;
      in[i] = e < n;
      idx[i] = in[i] ? e * nrhs + r : r;  // past the end: entry 0, in bounds, not stored
      acc[i] = w[idx[i]];
    }
    if (ok) {
      // w^ = w - sum_j c_j W_j, oldest direction first; four directions of all
      // entries in flight together
      constexpr int kU = 4;
      for (int j0 = 0; j0 < nj; j0 += kU) {
        C wl[kU][kE];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int64_t off = int64_t(min(j0 + u, nj - 1)) * fstride;
#pragma unroll
          for (int i = 0; i < kE; ++i) wl[u][i] = Wb[off + idx[i]];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          if (j0 + u < nj) {
            const double2 cd = cf[rl][j0 + u];
            const C cm = mk<C>(T(-cd.x), T(-cd.y));
#pragma unroll
            for (int i = 0; i < kE; ++i) cfma(acc[i], cm, wl[u][i]);
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kE; ++i) {
      if (!in[i]) continue;
      const C wn = cscale(acc[i], T(inv));
      w[idx[i]] = wn;
      C rr = res[idx[i]];
      if (ok) {
        const C aw = cmul(ar, wn);
        rr.x -= aw.x;
        rr.y -= aw.y;
        res[idx[i]] = rr;
      }
      racc += double(rr.x) * rr.x + double(rr.y) * rr.y;
    }
  }
  __syncthreads();  // sh is reused
  if (l < 64) sh[l][rl][0] = racc;
  __syncthreads();
  if (t < rg) {
    double a = 0;
    for (int k = 0; k < 64; ++k) a += sh[k][t][0];
    partial[int64_t(blockIdx.x) * nrhs + r0 + t] = a;
  }
}

// Coefficients of the solution over the unmodified directions z_i of a lazy
// inner solve (one wavefront per RHS, lane j holding coefficient j).  The GCR
// direction is p_i = inv_i (z_i - sum_{j<i} c_ij p_j) and x = sum_i a_i p_i;
// eliminating p from the last direction down gives x = sum_i d_i z_i with
// d_i = s_i inv_i and s_j -= d_i c_ij (j < i), s starting at a.
__global__ __launch_bounds__(64) void lazy_coef_kernel(const double2* __restrict__ hcoef,
                                                       const double* __restrict__ hinv,
                                                       const double2* __restrict__ ha, int K, int nrhs,
                                                       double2* __restrict__ dcoef) {
  const int r = blockIdx.x, j = threadIdx.x;
  double2 sj = j < K ? ha[int64_t(j) * nrhs + r] : make_double2(0, 0);
  double2 dj = make_double2(0, 0);
  for (int i = K - 1; i >= 0; --i) {
    const double inv = hinv[int64_t(i) * nrhs + r];
    const double dx = __shfl(sj.x * inv, i), dy = __shfl(sj.y * inv, i);
    if (j == i) dj = make_double2(dx, dy);
    if (j < i) {
      const double2 c = hcoef[(int64_t(i) * nrhs + r) * kMaxCoef + j];
      sj.x -= dx * c.x - dy * c.y;
      sj.y -= dx * c.y + dy * c.x;
    }
  }
  dcoef[int64_t(r) * kMaxCoef + j] = dj;
}

// x = sum_{i<K} d_i z_i (directions added in order).
template <class C>
__global__ __launch_bounds__(kT) void lazy_solution_kernel(const C* __restrict__ Zb, int64_t fstride, int K,
                                                           const double2* __restrict__ dcoef, C* __restrict__ x,
                                                           int64_t n, int nrhs, int64_t rs, int64_t es) {
  constexpr int kU = 4;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * nrhs) return;
  const int r = es == 1 ? int(t / n) : int(t % nrhs);
  const int64_t idx = int64_t(r) * rs + (es == 1 ? t % n : t / nrhs) * es;
  using T = decltype(C::x);
  C xx = mk<C>(T(0), T(0));
  for (int i0 = 0; i0 < K; i0 += kU) {
    C zl[kU], c[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u < K ? i0 + u : K - 1;  // past the end: the last direction (in bounds), not added
      const double2 d = dcoef[int64_t(r) * kMaxCoef + i];
      c[u] = mk<C>(T(d.x), T(d.y));
      zl[u] = Zb[int64_t(i) * fstride + idx];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (i0 + u < K) cfma(xx, c[u], zl[u]);
  }
  x[idx] = xx;
}

// The same elimination for the outer solve, whose directions sit in a ring of
// nslots slots shared by all RHS: RHS r's current cycle is the window of its
// nb[r] latest directions, ending at ring slot last.  Per-direction records
// are indexed [slot][cap] (c: [slot][cap][kMaxCoef] over ring slots); only
// the a_i not yet applied are non-zero, and they are cleared once applied.
__global__ __launch_bounds__(64) void ring_lazy_coef_kernel(const double2* __restrict__ hcoef,
                                                            const double* __restrict__ hinv,
                                                            double2* __restrict__ ha, const int* __restrict__ nb,
                                                            int last, int nslots, int cap,
                                                            double2* __restrict__ dcoef) {
  const int r = blockIdx.x, k = threadIdx.x, n = nb[r];
  const int sk = (last - n + 1 + k + 2 * nslots) % nslots;  // ring slot of window position k
  double2 s = k < n ? ha[int64_t(sk) * cap + r] : make_double2(0, 0);
  double2 d = make_double2(0, 0);
  for (int i = n - 1; i >= 0; --i) {
    const int si = (last - n + 1 + i + 2 * nslots) % nslots;
    const double inv = hinv[int64_t(si) * cap + r];
    const double dx = __shfl(s.x * inv, i), dy = __shfl(s.y * inv, i);
    if (k == i) d = make_double2(dx, dy);
    if (k < i) {
      const double2 c = hcoef[(int64_t(si) * cap + r) * kMaxCoef + sk];
      s.x -= dx * c.x - dy * c.y;
      s.y -= dx * c.y + dy * c.x;
    }
  }
  dcoef[int64_t(r) * kMaxCoef + k] = k < n ? d : make_double2(0, 0);
  if (k < n) ha[int64_t(sk) * cap + r] = make_double2(0, 0);
}

// x_r += sum_k d_k z_{slot k} over RHS r's window, oldest direction first (rhs-outer fields).
// The directions are stored as CZ: C itself, or float2 when they hold FP32
// values (widened exactly).
template <class C, class CZ>
__global__ __launch_bounds__(kT) void ring_lazy_x_kernel(const CZ* __restrict__ Zb, int64_t fstride,
                                                         const int* __restrict__ nb, int last, int nslots,
                                                         const double2* __restrict__ dcoef, C* __restrict__ x,
                                                         int64_t n, int nrhs, int64_t rs) {
  constexpr int kU = 4;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * nrhs) return;
  const int r = int(t / n);
  const int64_t idx = int64_t(r) * rs + t % n;
  const int m = nb[r];
  if (m == 0) return;
  using T = decltype(C::x);
  C xx = x[idx];
  for (int k0 = 0; k0 < m; k0 += kU) {
    C zl[kU], c[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = k0 + u < m ? k0 + u : m - 1;  // past the end: the last direction (in bounds), not added
      const int sk = (last - m + 1 + k + 2 * nslots) % nslots;
      const double2 d = dcoef[int64_t(r) * kMaxCoef + k];
      c[u] = mk<C>(T(d.x), T(d.y));
      const CZ zv = Zb[int64_t(sk) * fstride + idx];
      zl[u] = mk<C>(T(zv.x), T(zv.y));
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (k0 + u < m) cfma(xx, c[u], zl[u]);
  }
  x[idx] = xx;
}

// rn2[r] = sum of partials (wavefront g adds chunks g, g + 4, ... in order, then
// the four sums in a fixed order); convergence bookkeeping of an inner solve.
__global__ __launch_bounds__(kT) void check_kernel(const double* __restrict__ partial, int64_t nch, int nrhs,
                                                   double tol2, const double* __restrict__ b2,
                                                   const int* __restrict__ breakdown, int* __restrict__ active,
                                                   int* __restrict__ iters, double* __restrict__ rn2,
                                                   int* __restrict__ n_active, int* __restrict__ level_iters,
                                                   int* __restrict__ n_active_host) {
  __shared__ double sh[kT / 64][64];
  __shared__ int cnt;
  const int q = threadIdx.x & 63, g = threadIdx.x >> 6;
  if (threadIdx.x == 0) cnt = 0;
  for (int r0 = 0; r0 < nrhs; r0 += 64) {
    const int r = r0 + q;
    double acc = 0;
    if (r < nrhs) {
      // loads issued kRedLoads at a time, added in chunk order
      for (int64_t c0 = g; c0 < nch; c0 += kRedLoads * (kT / 64)) {
        double v[kRedLoads];
#pragma unroll
        for (int u = 0; u < kRedLoads; ++u) {
          const int64_t c = c0 + int64_t(u) * (kT / 64);
          v[u] = c < nch ? partial[c * nrhs + r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kRedLoads; ++u)
          if (c0 + int64_t(u) * (kT / 64) < nch) acc += v[u];
      }
    }
    sh[g][q] = acc;
    __syncthreads();
    if (g == 0 && r < nrhs) {
      const double s = ((sh[0][q] + sh[1][q]) + sh[2][q]) + sh[3][q];
      rn2[r] = s;
      if (active[r]) {
        iters[r] += 1;
        if (level_iters) level_iters[r] += 1;
        const bool bd = breakdown ? breakdown[r] != 0 : false;
        if (bd || !(s > tol2 * b2[r])) active[r] = 0;
      }
      if (active[r]) atomicAdd(&cnt, 1);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *n_active = cnt;
    if (n_active_host) *n_active_host = cnt;  // pinned host copy: the host polls it without a copy launch
  }
}

// Start of an inner solve: x = 0, r = b, b2 = ||b||^2 from sums3, active = b2 > 0, iters = 0.
__global__ void start_kernel(const double* __restrict__ sums3, int nrhs, double* __restrict__ b2,
                             int* __restrict__ active, int* __restrict__ iters, int* __restrict__ n_active) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int r = threadIdx.x; r < nrhs; r += blockDim.x) {
    const double s = sums3[3 * r + 2];
    b2[r] = s;
    active[r] = s > 0.0;
    iters[r] = 0;
    if (s > 0.0) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) *n_active = cnt;
}

// out = a x + b y (out may be y)
template <class C>
__global__ __launch_bounds__(kT) void axpby_kernel(const C* __restrict__ x, const C* y, C* out, double a, double b,
                                                   int64_t total) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  using T = decltype(C::x);
  const C xv = x[i];
  C yv = b == 0.0 ? mk<C>(T(0), T(0)) : cscale(y[i], T(b));
  yv.x += T(a) * xv.x;
  yv.y += T(a) * xv.y;
  out[i] = yv;
}

// y[r] = x[r] for the RHS with mask[r] != 0 (fine or coarse layout)
template <class C>
__global__ __launch_bounds__(kT) void masked_copy_kernel(const C* __restrict__ x, C* __restrict__ y,
                                                         const int* __restrict__ mask, int64_t n, int nrhs, int64_t rs,
                                                         int64_t es) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * nrhs) return;
  const int r = es == 1 ? int(t / n) : int(t % nrhs);
  if (!mask[r]) return;
  const int64_t e = es == 1 ? t % n : t / nrhs;
  const int64_t idx = int64_t(r) * rs + e * es;
  y[idx] = x[idx];
}

}  // namespace

int64_t gcr_partial_rows(int64_t n, bool inner) {
  const int64_t c = chunk_for_shape(n, inner);
  return (n + c - 1) / c;
}

namespace {
// Chunks of the per-RHS partial sums of a field shape (see the kernels).
int64_t shape_chunks(const FieldShape& f) { return gcr_partial_rows(f.n, f.es != 1); }

template <class C>
void launch_multidot(int nc, int64_t nch, const FieldShape& f, const C* W, int64_t fstride, const C* w, int64_t chunk,
                     double* partial, const uint32_t* valid, int vbit0, hipStream_t st) {
  auto grid = [&](int G) { return dim3(unsigned(nch), unsigned(f.nrhs), unsigned((nc + G - 1) / G)); };
  if (nc <= 4)
    hipLaunchKernelGGL((multidot_kernel<C, 4>), grid(4), dim3(kT), 0, st, W, fstride, nc, w, f.n, f.nrhs, f.rs, f.es,
                       chunk, partial, valid, vbit0);
  else if (nc <= 8)
    hipLaunchKernelGGL((multidot_kernel<C, 8>), grid(8), dim3(kT), 0, st, W, fstride, nc, w, f.n, f.nrhs, f.rs, f.es,
                       chunk, partial, valid, vbit0);
  else
    hipLaunchKernelGGL((multidot_kernel<C, 16>), grid(16), dim3(kT), 0, st, W, fstride, nc, w, f.n, f.nrhs, f.rs,
                       f.es, chunk, partial, valid, vbit0);
}
}  // namespace

void gcr_multidot(int prec, const void* W, int64_t fstride, int nj, const void* w, const FieldShape& f, double* partial,
                  const uint32_t* valid, double2* coef, hipStream_t st) {
  if (nj <= 0) return;
  CRK_REQUIRE(nj <= kMaxCoef, "GCR basis above 64 vectors");
  CRK_REQUIRE(valid == nullptr || nj <= 32, "masked GCR basis above 32 vectors");
  const int64_t chunk = chunk_for_shape(f.n, f.es != 1), nch = shape_chunks(f);
  const size_t esz = prec == CRK_FORM_FP64 ? sizeof(double2) : sizeof(float2);
  for (int j0 = 0; j0 < nj; j0 += kMaxBasis) {
    const int nc = nj - j0 < kMaxBasis ? nj - j0 : kMaxBasis;
    const unsigned ng = unsigned((nc + kDotGroup - 1) / kDotGroup);
    const dim3 g = dim3(unsigned(nch), unsigned(f.nrhs), ng), gi = g;
    const void* Wj = static_cast<const char*>(W) + esz * size_t(j0) * size_t(fstride);
    const bool rhs_inner = f.es != 1 && f.rs == 1 && f.es == f.nrhs;
    const dim3 grg = dim3(unsigned(nch), unsigned((f.nrhs + kInnerRhs - 1) / kInnerRhs),
                          unsigned((nc + kInnerGroup - 1) / kInnerGroup));
    const dim3 brg = dim3(unsigned(64 * std::min(f.nrhs, kInnerRhs)));
    if (rhs_inner && prec == CRK_FORM_FP64)
      hipLaunchKernelGGL(multidot_inner_rg_kernel<double2>, grg, brg, 0, st, static_cast<const double2*>(Wj),
                         fstride, nc, static_cast<const double2*>(w), f.n, f.nrhs, partial);
    else if (rhs_inner)
      hipLaunchKernelGGL(multidot_inner_rg_kernel<float2>, grg, brg, 0, st, static_cast<const float2*>(Wj),
                         fstride, nc, static_cast<const float2*>(w), f.n, f.nrhs, partial);
    else if (f.es != 1 && prec == CRK_FORM_FP64)
      hipLaunchKernelGGL(multidot_inner_kernel<double2>, gi, dim3(64), 0, st, static_cast<const double2*>(Wj), fstride,
                         nc, static_cast<const double2*>(w), f.n, f.nrhs, f.rs, f.es, partial);
    else if (f.es != 1)
      hipLaunchKernelGGL(multidot_inner_kernel<float2>, gi, dim3(64), 0, st, static_cast<const float2*>(Wj), fstride,
                         nc, static_cast<const float2*>(w), f.n, f.nrhs, f.rs, f.es, partial);
    else if (prec == CRK_FORM_FP64)
      launch_multidot<double2>(nc, nch, f, static_cast<const double2*>(Wj), fstride, static_cast<const double2*>(w),
                               chunk, partial, valid, j0, st);
    else
      launch_multidot<float2>(nc, nch, f, static_cast<const float2*>(Wj), fstride, static_cast<const float2*>(w),
                              chunk, partial, valid, j0, st);
    CRK_LAUNCH_CHECK();
    hipLaunchKernelGGL(multidot_reduce_kernel, dim3(unsigned(f.nrhs)), dim3(kT), 0, st, partial, nch, f.nrhs, j0, nc,
                       valid, coef);
    CRK_LAUNCH_CHECK();
  }
}

void gcr_multiaxpy_w(int prec, const void* W, int64_t fstride, int nj, int j_first, void* w, const double2* coef,
                     const FieldShape& f, hipStream_t st) {
  if (nj <= 0) return;
  CRK_REQUIRE(nj <= kMaxCoef, "GCR basis above 64 vectors");
  CRK_REQUIRE(j_first >= 0 && j_first < nj, "GCR ring start out of range");
  const dim3 g(ceil_div(f.n * f.nrhs, kT));
  if (prec == CRK_FORM_FP64)
    hipLaunchKernelGGL(multiaxpy_kernel<double2>, g, dim3(kT), 0, st, static_cast<const double2*>(W), fstride, nj,
                       j_first, static_cast<double2*>(w), coef, f.n, f.nrhs, f.rs, f.es);
  else
    hipLaunchKernelGGL(multiaxpy_kernel<float2>, g, dim3(kT), 0, st, static_cast<const float2*>(W), fstride, nj,
                       j_first, static_cast<float2*>(w), coef, f.n, f.nrhs, f.rs, f.es);
  CRK_LAUNCH_CHECK();
}

void gcr_update_lazy(int prec, void* w, void* r, const double* dpart, int64_t dnch, const int* active, int* breakdown,
                     const FieldShape& f, double* partial, double* rn2, double* hinv, double2* ha, hipStream_t st) {
  const int64_t nch = shape_chunks(f);
  if (!(f.es != 1 && f.rs == 1 && f.es == f.nrhs)) {  // one RHS, or rhs-outer: the per-RHS kernel
    const int64_t chunk = chunk_for_shape(f.n, f.es != 1);
    const dim3 g = dim3(unsigned(nch), unsigned(f.nrhs));
    if (prec == CRK_FORM_FP64)
      hipLaunchKernelGGL(update_fused_kernel<double2>, g, dim3(kT), 0, st, static_cast<double2*>(w),
                         static_cast<double2*>(r), dpart, dnch, active, breakdown, f.n, f.nrhs, f.rs, f.es, chunk,
                         partial, hinv, ha);
    else
      hipLaunchKernelGGL(update_fused_kernel<float2>, g, dim3(kT), 0, st, static_cast<float2*>(w),
                         static_cast<float2*>(r), dpart, dnch, active, breakdown, f.n, f.nrhs, f.rs, f.es, chunk,
                         partial, hinv, ha);
    CRK_LAUNCH_CHECK();
    if (rn2) reduce_partials(partial, nch, f.nrhs, 1, rn2, st);
    return;
  }
  const dim3 grg = dim3(unsigned(nch), unsigned((f.nrhs + kInnerRhs - 1) / kInnerRhs));
  const dim3 brg = dim3(unsigned(64 * std::min(f.nrhs, kInnerRhs)));
  if (prec == CRK_FORM_FP64)
    hipLaunchKernelGGL(update_fused_rg_kernel<double2>, grg, brg, 0, st, static_cast<double2*>(w),
                       static_cast<double2*>(r), dpart, dnch, active, breakdown, f.n, f.nrhs, partial, hinv, ha);
  else
    hipLaunchKernelGGL(update_fused_rg_kernel<float2>, grg, brg, 0, st, static_cast<float2*>(w),
                       static_cast<float2*>(r), dpart, dnch, active, breakdown, f.n, f.nrhs, partial, hinv, ha);
  CRK_LAUNCH_CHECK();
  if (rn2) reduce_partials(partial, nch, f.nrhs, 1, rn2, st);
}

bool gcr_one_pass_shape(const FieldShape& f) { return f.rs == 1 && f.es == f.nrhs; }

int64_t gcr_gs_update(int prec, const void* W, int64_t fstride, int nj, void* w, void* r, const double2* coef,
                   const double* dpart, int64_t dnch, const int* active, int* breakdown, const FieldShape& f,
                   double* partial, double* hinv, double2* ha, hipStream_t st) {
  CRK_REQUIRE(gcr_one_pass_shape(f), "one-pass GCR step: rhs-inner fields only");
  CRK_REQUIRE(nj >= 0 && nj <= kMaxCoef, "one-pass GCR step: 0 <= directions <= 64");
  const int64_t nch = gcr_partial_rows(f.n, true);  // one RHS too: the same chunks as for many
  const dim3 g = dim3(unsigned(nch), unsigned((f.nrhs + kInnerRhs - 1) / kInnerRhs));
  const dim3 b = dim3(unsigned(64 * std::min(f.nrhs, kInnerRhs)));
  if (prec == CRK_FORM_FP64)
    hipLaunchKernelGGL(gs_update_rg_kernel<double2>, g, b, 0, st, static_cast<const double2*>(W), fstride, nj,
                       static_cast<double2*>(w), static_cast<double2*>(r), coef, dpart, dnch, active, breakdown, f.n,
                       f.nrhs, partial, hinv, ha, 1e-13);
  else
    hipLaunchKernelGGL(gs_update_rg_kernel<float2>, g, b, 0, st, static_cast<const float2*>(W), fstride, nj,
                       static_cast<float2*>(w), static_cast<float2*>(r), coef, dpart, dnch, active, breakdown, f.n,
                       f.nrhs, partial, hinv, ha, 1e-6);
  CRK_LAUNCH_CHECK();
  return nch;
}

void gcr_gs_update_ring(int prec, const void* W, int64_t fstride, int nj, int j_first, void* w, void* r,
                        const double2* coef, const double* dpart, int64_t dnch, const int* active, int* breakdown,
                        const FieldShape& f, double* partial, double* rn2, double* hinv, double2* ha, hipStream_t st) {
  CRK_REQUIRE(f.es == 1, "one-pass ring step: rhs-outer fields only");
  CRK_REQUIRE(nj >= 0 && nj <= kMaxCoef && j_first >= 0 && (nj == 0 || j_first < nj), "one-pass ring step: bad ring");
  const int64_t nch = shape_chunks(f), chunk = chunk_for_shape(f.n, false);
  const dim3 g = dim3(unsigned(nch), unsigned(f.nrhs));
  if (prec == CRK_FORM_FP64)
    hipLaunchKernelGGL(gs_update_ring_kernel<double2>, g, dim3(kT), 0, st, static_cast<const double2*>(W), fstride,
                       nj, j_first, static_cast<double2*>(w), static_cast<double2*>(r), coef, dpart, dnch, active,
                       breakdown, f.n, f.nrhs, f.rs, chunk, partial, hinv, ha, 1e-13);
  else
    hipLaunchKernelGGL(gs_update_ring_kernel<float2>, g, dim3(kT), 0, st, static_cast<const float2*>(W), fstride,
                       nj, j_first, static_cast<float2*>(w), static_cast<float2*>(r), coef, dpart, dnch, active,
                       breakdown, f.n, f.nrhs, f.rs, chunk, partial, hinv, ha, 1e-6);
  CRK_LAUNCH_CHECK();
  if (rn2) reduce_partials(partial, nch, f.nrhs, 1, rn2, st);
}

void gcr_lazy_solution(int prec, const void* Z, int64_t fstride, int K, void* x, const double2* hcoef,
                       const double* hinv, const double2* ha, double2* dcoef, const FieldShape& f, hipStream_t st) {
  CRK_REQUIRE(K >= 1 && K <= kMaxCoef, "lazy GCR solution: 1 <= K <= 64 directions");
  hipLaunchKernelGGL(lazy_coef_kernel, dim3(unsigned(f.nrhs)), dim3(64), 0, st, hcoef, hinv, ha, K, f.nrhs, dcoef);
  CRK_LAUNCH_CHECK();
  const dim3 g(ceil_div(f.n * f.nrhs, kT));
  if (prec == CRK_FORM_FP64)
    hipLaunchKernelGGL(lazy_solution_kernel<double2>, g, dim3(kT), 0, st, static_cast<const double2*>(Z), fstride, K,
                       dcoef, static_cast<double2*>(x), f.n, f.nrhs, f.rs, f.es);
  else
    hipLaunchKernelGGL(lazy_solution_kernel<float2>, g, dim3(kT), 0, st, static_cast<const float2*>(Z), fstride, K,
                       dcoef, static_cast<float2*>(x), f.n, f.nrhs, f.rs, f.es);
  CRK_LAUNCH_CHECK();
}

void gcr_ring_materialize(const void* Z, int z_form, int64_t fstride, const int* nb, int last, int nslots, int cap,
                          void* x, const double2* hcoef, const double* hinv, double2* ha, double2* dcoef,
                          const FieldShape& f, hipStream_t st) {
  CRK_REQUIRE(f.es == 1, "ring materialisation: rhs-outer fields only");
  CRK_REQUIRE(nslots >= 1 && nslots <= kMaxCoef && f.nrhs <= cap, "ring materialisation: bad ring");
  CRK_REQUIRE(z_form == CRK_FORM_FP64 || z_form == CRK_FORM_FP32, "ring materialisation: directions FP64 or FP32");
  hipLaunchKernelGGL(ring_lazy_coef_kernel, dim3(unsigned(f.nrhs)), dim3(64), 0, st, hcoef, hinv, ha, nb, last, nslots,
                     cap, dcoef);
  CRK_LAUNCH_CHECK();
  const dim3 g(ceil_div(f.n * f.nrhs, kT));
  if (z_form == CRK_FORM_FP64)
    hipLaunchKernelGGL((ring_lazy_x_kernel<double2, double2>), g, dim3(kT), 0, st, static_cast<const double2*>(Z),
                       fstride, nb, last, nslots, dcoef, static_cast<double2*>(x), f.n, f.nrhs, f.rs);
  else
    hipLaunchKernelGGL((ring_lazy_x_kernel<double2, float2>), g, dim3(kT), 0, st, static_cast<const float2*>(Z),
                       fstride, nb, last, nslots, dcoef, static_cast<double2*>(x), f.n, f.nrhs, f.rs);
  CRK_LAUNCH_CHECK();
}

void gcr_check(const double* partial, const FieldShape& f, double tol2, const double* b2, const int* breakdown,
               int* active, int* iters, double* rn2, int* n_active, int* level_iters, hipStream_t st,
               int* n_active_host, int64_t partial_rows) {
  const int64_t nch = partial_rows >= 0 ? partial_rows : shape_chunks(f);
  hipLaunchKernelGGL(check_kernel, dim3(1), dim3(kT), 0, st, partial, nch, f.nrhs, tol2, b2, breakdown, active, iters,
                     rn2, n_active, level_iters, n_active_host);
  CRK_LAUNCH_CHECK();
}

void gcr_start(const double* sums3, int nrhs, double* b2, int* active, int* iters, int* n_active, hipStream_t st) {
  hipLaunchKernelGGL(start_kernel, dim3(1), dim3(64), 0, st, sums3, nrhs, b2, active, iters, n_active);
  CRK_LAUNCH_CHECK();
}

void field_axpby_to(int prec, const void* x, const void* y, void* out, double a, double b, int64_t total,
                    hipStream_t st) {
  if (total <= 0) return;
  const dim3 g(ceil_div(total, kT));
  if (prec == CRK_FORM_FP64)
    hipLaunchKernelGGL(axpby_kernel<double2>, g, dim3(kT), 0, st, static_cast<const double2*>(x),
                       static_cast<const double2*>(y), static_cast<double2*>(out), a, b, total);
  else
    hipLaunchKernelGGL(axpby_kernel<float2>, g, dim3(kT), 0, st, static_cast<const float2*>(x),
                       static_cast<const float2*>(y), static_cast<float2*>(out), a, b, total);
  CRK_LAUNCH_CHECK();
}

void field_axpby(int prec, const void* x, void* y, double a, double b, int64_t total, hipStream_t st) {
  field_axpby_to(prec, x, y, y, a, b, total, st);
}

void field_masked_copy(int prec, const void* x, void* y, const int* mask, const FieldShape& f, hipStream_t st) {
  const dim3 g(ceil_div(f.n * f.nrhs, kT));
  if (prec == CRK_FORM_FP64)
    hipLaunchKernelGGL(masked_copy_kernel<double2>, g, dim3(kT), 0, st, static_cast<const double2*>(x),
                       static_cast<double2*>(y), mask, f.n, f.nrhs, f.rs, f.es);
  else
    hipLaunchKernelGGL(masked_copy_kernel<float2>, g, dim3(kT), 0, st, static_cast<const float2*>(x),
                       static_cast<float2*>(y), mask, f.n, f.nrhs, f.rs, f.es);
  CRK_LAUNCH_CHECK();
}

}  // namespace crk
