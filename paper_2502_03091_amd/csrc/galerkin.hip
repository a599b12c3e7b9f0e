// Galerkin coarse operator D_c = P^dag D P of the fine Wilson operator
// (paper, Sec. 2, Eq. (4); P block diagonal with chirality-sparse blocks, Eq. (6)).
//
// With P(x) the 12 x 2k block of P at fine site x and H_{+-mu}(x) the Wilson hops
// -w_mu/2 (1 -+ gamma_mu) (x) U:
//   X(j)       = sum_{x in block j} P(x)^dag [ (m0 + sum w) P(x) + sum_{in-block hops} H P(x+-mu) ]
//                (with the clover term the site term is the block diagonal diag 1 + C(x))
//   Y_{+mu}(j) = sum_{x in block j, x+mu outside} P(x)^dag H_{+mu}(x) P(x+mu)
//   Y_{-mu}(j) = sigma3 Y_{+mu}(j-mu)^dag sigma3          (gamma5-hermiticity of D)
// One workgroup per (coarse site, part) with part 0 = X and parts 1..4 = Y_{+mu}.
// For each fine site the hop results T = sum H P(y) (12 x 2k) are formed by
// threads (site of a batch, column), each for all three colours, from the
// half-spinor projection, staged in LDS, and contracted with P(x)^dag into
// per-thread register tiles of the 2k x 2k output.
// Coarse links are stored per coarse site as 9 column-major 2k x 2k blocks:
// index 0 = X, 1 + 2mu = Y_{+mu}, 2 + 2mu = Y_{-mu}.
#include "field.h"
#include "galerkin.h"

namespace crk {

namespace {

constexpr int kT = 256;
constexpr int kGalerkinMaxNb = 1024;  // fine sites per block (list in LDS)

// Projection of the (chirality-sparse) column onto the half spinor of (1 - sign gamma_mu).
template <int MU, int SIGN>
__device__ __forceinline__ void project_col(const double2 (&s)[4][3], double2 (&h)[2][3]) {
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const double2 s0 = s[0][b], s1 = s[1][b], s2 = s[2][b], s3 = s[3][b];
    if constexpr (MU == 0) {
      if constexpr (SIGN > 0) { h[0][b] = s0 + cmuli(s3); h[1][b] = s1 + cmuli(s2); }
      else { h[0][b] = s0 - cmuli(s3); h[1][b] = s1 - cmuli(s2); }
    } else if constexpr (MU == 1) {
      if constexpr (SIGN > 0) { h[0][b] = s0 + s3; h[1][b] = s1 - s2; }
      else { h[0][b] = s0 - s3; h[1][b] = s1 + s2; }
    } else if constexpr (MU == 2) {
      if constexpr (SIGN > 0) { h[0][b] = s0 + cmuli(s2); h[1][b] = s1 - cmuli(s3); }
      else { h[0][b] = s0 - cmuli(s2); h[1][b] = s1 + cmuli(s3); }
    } else {
      if constexpr (SIGN > 0) { h[0][b] = s0 - s2; h[1][b] = s1 - s3; }
      else { h[0][b] = s0 + s2; h[1][b] = s1 + s3; }
    }
  }
}

// t[spin] += coef * rebuilt spinor (colour a) from g0, g1.
template <int MU, int SIGN>
__device__ __forceinline__ void rebuild(double2 (&t)[4], double2 g0, double2 g1, double coef) {
  double2 l2, l3;
  if constexpr (MU == 0) {
    if constexpr (SIGN > 0) { l2 = cscale(cmuli(g1), -1.0); l3 = cscale(cmuli(g0), -1.0); }
    else { l2 = cmuli(g1); l3 = cmuli(g0); }
  } else if constexpr (MU == 1) {
    if constexpr (SIGN > 0) { l2 = cscale(g1, -1.0); l3 = g0; }
    else { l2 = g1; l3 = cscale(g0, -1.0); }
  } else if constexpr (MU == 2) {
    if constexpr (SIGN > 0) { l2 = cscale(cmuli(g0), -1.0); l3 = cmuli(g1); }
    else { l2 = cmuli(g0); l3 = cscale(cmuli(g1), -1.0); }
  } else {
    if constexpr (SIGN > 0) { l2 = cscale(g0, -1.0); l3 = cscale(g1, -1.0); }
    else { l2 = g0; l3 = g1; }
  }
  t[0] = t[0] + cscale(g0, coef);
  t[1] = t[1] + cscale(g1, coef);
  t[2] = t[2] + cscale(l2, coef);
  t[3] = t[3] + cscale(l3, coef);
}

// P(y)[:, col] as a 4x3 spinor (zero outside the column's chirality).
__device__ __forceinline__ void load_pcol(const GalerkinArgs& A, int64_t y, int col, double2 (&s)[4][3]) {
  const int k = A.k, beta = col / k, i = col % k;
  const int64_t jy = y / A.nb, ly = y % A.nb;
  const double2* p = A.P + ((2 * jy + beta) * k + i) * int64_t(A.nr) + ly;
  const double2 z = make_double2(0, 0);
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double2 v = p[int64_t(3 * sp + b) * A.nb];
      s[sp][b] = beta == 0 ? v : z;       // constant indices only: no local-memory arrays
      s[2 + sp][b] = beta == 0 ? z : v;
    }
}

template <int MU, int SIGN>
__device__ __forceinline__ void add_hop(const GalerkinArgs& A, int64_t x, int64_t y, int col, double2 (&t)[3][4]) {
  double2 s[4][3], h[2][3];
  load_pcol(A, y, col, s);
  project_col<MU, SIGN>(s, h);
  const int64_t Vp = pad_sites(A.V);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double2 g0 = make_double2(0, 0), g1 = make_double2(0, 0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if constexpr (SIGN > 0) {
        const double2 u = A.gauge[aidx(MU, 3 * a + b, x, Vp, 9)];
        cfma(g0, u, h[0][b]);
        cfma(g1, u, h[1][b]);
      } else {
        const double2 u = A.gauge[aidx(MU, 3 * b + a, y, Vp, 9)];
        cfmac(g0, u, h[0][b]);
        cfmac(g1, u, h[1][b]);
      }
    }
    rebuild<MU, SIGN>(t[a], g0, g1, A.hw[MU]);
  }
}

template <int MU, int SIGN>
__device__ __forceinline__ void maybe_hop(const GalerkinArgs& A, int64_t x, int64_t j, int col, int part,
                                          double2 (&t)[3][4]) {
  const int64_t y = A.nbr[int64_t(2 * MU + (SIGN > 0 ? 0 : 1)) * A.V + x];
  const bool inside = (y / A.nb) == j;
  if (part == 0 ? inside : (SIGN > 0 && MU == part - 1 && !inside)) add_hop<MU, SIGN>(A, x, y, col, t);
}

// The block's contributing sites (all for X, the +mu face for Y_{+mu}) are
// listed in site order and taken kSiteBatch at a time: the hop results of a
// batch are formed together, then added site by site in list order, so every
// output has the same summation order as a site-by-site loop.
constexpr int kSiteBatch = 5;

template <int TI>
__global__ __launch_bounds__(kT) void galerkin_kernel(GalerkinArgs A) {
  constexpr int N = 16 * TI;  // 2k
  // at 2k = 64 five sites would take 96 KB of LDS and leave one workgroup per
  // CU; four keep two (the summation order does not depend on the batch)
  constexpr int S = TI == 4 ? 4 : kSiteBatch;
  __shared__ double2 T[S][12][N];
  __shared__ double2 Pc[S][6][N];
  __shared__ int list[kGalerkinMaxNb];
  __shared__ int wcount[kT / 64];
  __shared__ int nlist;
  const int64_t j = blockIdx.x / 5;
  const int part = blockIdx.x % 5;
  const int k = A.k;
  const int rg = threadIdx.x / 16, cg = threadIdx.x % 16;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // compaction of the contributing local sites, in order
  if (threadIdx.x == 0) nlist = 0;
  for (int l0 = 0; l0 < A.nb; l0 += kT) {
    const int l = l0 + threadIdx.x;
    bool use = l < A.nb;
    if (use && part > 0) {
      const int64_t y = A.nbr[int64_t(2 * (part - 1)) * A.V + j * A.nb + l];
      use = (y / A.nb) != j;
    }
    const uint64_t m = __ballot(use);
    __syncthreads();
    if (lane == 0) wcount[wid] = __popcll(m);
    __syncthreads();
    int off = nlist;
    for (int w = 0; w < wid; ++w) off += wcount[w];
    if (use) list[off + __popcll(m & ((uint64_t(1) << lane) - 1))] = l;
    __syncthreads();
    if (threadIdx.x == 0) nlist += wcount[0] + wcount[1] + wcount[2] + wcount[3];
    __syncthreads();
  }
  const int nl = nlist;
  double2 acc[TI][TI];
#pragma unroll
  for (int x = 0; x < TI; ++x)
#pragma unroll
    for (int y = 0; y < TI; ++y) acc[x][y] = make_double2(0, 0);

  for (int b0 = 0; b0 < nl; b0 += S) {
    const int ns = min(S, nl - b0);
    __syncthreads();
    // P(x) per column, compressed to its chirality's 6 components
    for (int e = threadIdx.x; e < ns * 6 * N; e += blockDim.x) {
      const int sb = e / (6 * N), c = (e / N) % 6, col = e % N, beta = col / k, i = col % k;
      const int l = list[b0 + sb];
      Pc[sb][c][col] = A.P[((2 * j + beta) * k + i) * int64_t(A.nr) + int64_t(c) * A.nb + l];
    }
    // one thread per (site, column) forms the column's three colour rows, so
    // P(y) is read once per hop for all of them
    for (int e = threadIdx.x; e < ns * N; e += blockDim.x) {
      const int sb = e % ns, col = e / ns;  // the batch's sites side by side: their P(y) rows are adjacent
      const int l = list[b0 + sb];
      const int64_t x = j * A.nb + l;
      double2 t[3][4];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) t[a][sp] = make_double2(0, 0);
      if (part == 0) {
        // site term: (m0 + sum w) P(x), or with the clover term the site block
        // X_beta(x) (6 x 6) of the column's chirality times P(x)'s six rows
        const int beta = col / k, i = col % k;
        const double2* p = A.P + ((2 * j + beta) * k + i) * int64_t(A.nr) + l;
        const double2 z = make_double2(0, 0);
        double2 sv[6];
        if (A.clover) {
          double2 pc[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) pc[c] = p[int64_t(c) * A.nb];
          const double2* X = A.clover + aidx(0, 36 * beta, x, pad_sites(A.V), 72);
#pragma unroll
          for (int r = 0; r < 6; ++r) {
            double2 acc = z;
#pragma unroll
            for (int c = 0; c < 6; ++c) cfma(acc, X[(6 * r + c) * kVL], pc[c]);
            sv[r] = acc;
          }
        } else {
#pragma unroll
          for (int c = 0; c < 6; ++c) sv[c] = cscale(p[int64_t(c) * A.nb], A.diag);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const double2 v0 = sv[a], v1 = sv[3 + a];
          t[a][0] = beta == 0 ? v0 : z;
          t[a][1] = beta == 0 ? v1 : z;
          t[a][2] = beta == 0 ? z : v0;
          t[a][3] = beta == 0 ? z : v1;
        }
      }
      maybe_hop<0, +1>(A, x, j, col, part, t);
      maybe_hop<0, -1>(A, x, j, col, part, t);
      maybe_hop<1, +1>(A, x, j, col, part, t);
      maybe_hop<1, -1>(A, x, j, col, part, t);
      maybe_hop<2, +1>(A, x, j, col, part, t);
      maybe_hop<2, -1>(A, x, j, col, part, t);
      maybe_hop<3, +1>(A, x, j, col, part, t);
      maybe_hop<3, -1>(A, x, j, col, part, t);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) T[sb][3 * sp + a][col] = t[a][sp];
    }
    __syncthreads();
    // acc[r][c] += sum_c' conj(P(x)[alpha_r*6 + c'][r]) T[alpha_r*6 + c'][c], sites in list order
    for (int sb = 0; sb < ns; ++sb) {
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        // this thread's T columns of both chiralities, read once for all TI rows
        double2 t0[TI], t1[TI];
#pragma unroll
        for (int yc = 0; yc < TI; ++yc) {
          t0[yc] = T[sb][c][cg * TI + yc];
          t1[yc] = T[sb][6 + c][cg * TI + yc];
        }
#pragma unroll
        for (int xr = 0; xr < TI; ++xr) {
          const int r = rg * TI + xr;
          const bool ar = r >= k;
          const double2 pr = Pc[sb][c][r];
#pragma unroll
          for (int yc = 0; yc < TI; ++yc) cfmac(acc[xr][yc], pr, ar ? t1[yc] : t0[yc]);
        }
      }
    }
  }
  // store column-major: link[jpos][part == 0 ? 0 : 1 + 2mu][col][row]
  const int64_t jpos = A.pos_c ? A.pos_c[j] : j;
  const int nbidx = part == 0 ? 0 : 1 + 2 * (part - 1);
  double2* out = A.links + (jpos * 9 + nbidx) * int64_t(N) * N;
#pragma unroll
  for (int xr = 0; xr < TI; ++xr)
#pragma unroll
    for (int yc = 0; yc < TI; ++yc) {
      const int r = rg * TI + xr, c = cg * TI + yc;
      out[int64_t(c) * N + r] = acc[xr][yc];
    }
}

// Y_{-mu}(j) = sigma3 Y_{+mu}(j - mu)^dag sigma3 on the coarse lattice (device positions).
__global__ __launch_bounds__(kT) void backward_links_kernel(double2* __restrict__ links, const int* __restrict__ nbr_c,
                                                            int64_t Vc, int N, int k) {
  const int64_t jpos = blockIdx.x / 4;
  const int mu = blockIdx.x % 4;
  const int64_t jm = nbr_c[int64_t(2 * mu + 1) * Vc + jpos];
  const double2* src = links + (jm * 9 + 1 + 2 * mu) * int64_t(N) * N;
  double2* dst = links + (jpos * 9 + 2 + 2 * mu) * int64_t(N) * N;
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
    const int c = e / N, r = e % N;  // dst element (r, c), column-major
    const double sgn = ((r < k) == (c < k)) ? 1.0 : -1.0;
    const double2 v = src[int64_t(r) * N + c];  // src element (c, r)
    dst[int64_t(c) * N + r] = make_double2(sgn * v.x, -sgn * v.y);
  }
}

}  // namespace

void galerkin_fine(const GalerkinArgs& A, const int* nbr_c, int64_t Vc, hipStream_t st) {
  const int N = 2 * A.k;
  CRK_REQUIRE(N % 16 == 0 && N <= 128, "2k must be a multiple of 16 and <= 128");
  CRK_REQUIRE(A.nb >= 1 && A.nb <= kGalerkinMaxNb, "Galerkin: at most 1024 fine sites per block");
  const dim3 g = dim3(unsigned(A.ncoarse * 5));
  switch (N / 16) {
    case 1: hipLaunchKernelGGL(galerkin_kernel<1>, g, dim3(kT), 0, st, A); break;
    case 2: hipLaunchKernelGGL(galerkin_kernel<2>, g, dim3(kT), 0, st, A); break;
    case 3: hipLaunchKernelGGL(galerkin_kernel<3>, g, dim3(kT), 0, st, A); break;
    case 4: hipLaunchKernelGGL(galerkin_kernel<4>, g, dim3(kT), 0, st, A); break;
    default: fail(CRK_EINVAL, "2k above 64 is not supported by the Galerkin kernel");
  }
  CRK_LAUNCH_CHECK();
  hipLaunchKernelGGL(backward_links_kernel, dim3(unsigned(Vc * 4)), dim3(kT), 0, st, A.links, nbr_c, Vc, N, A.k);
  CRK_LAUNCH_CHECK();
}

}  // namespace crk

// ---------------------------------------------------------------- coarse levels
// Galerkin product of a coarse stencil operator (level l >= 1, N = 2h
// components per site, links [V][9][N][N] column-major) with its prolongator:
// the same X / Y_{+mu} formulas with the Wilson hops replaced by the stored
// link blocks, P(x) being chirality-sparse (rows alpha*h.. of column alpha*k+i).
namespace crk {
namespace {

template <int TI>
__global__ __launch_bounds__(256) void galerkin_coarse_kernel(GalerkinCoarseArgs A) {
  constexpr int NC = 16 * TI;  // 2k of the new level
  extern __shared__ double2 sm[];
  const int N = A.N, h = N / 2, k = A.k;
  double2* T = sm;             // [N][NC]  sum of link * P(y)
  double2* Pc = T + N * NC;    // [h][NC]  P(x) compressed to its chirality's h rows
  const int64_t j = blockIdx.x / 5;
  const int part = blockIdx.x % 5;
  const int rg = threadIdx.x / 16, cg = threadIdx.x % 16;
  double2 acc[TI][TI];
#pragma unroll
  for (int x = 0; x < TI; ++x)
#pragma unroll
    for (int y = 0; y < TI; ++y) acc[x][y] = make_double2(0, 0);
  for (int l = 0; l < A.nb; ++l) {
    const int64_t x = j * A.nb + l;
    if (part > 0) {
      const int64_t y = A.nbr[int64_t(2 * (part - 1)) * A.V + x];
      if (y / A.nb == j) continue;  // uniform across the workgroup
    }
    __syncthreads();
    for (int e = threadIdx.x; e < h * NC; e += blockDim.x) {
      const int c = e / NC, col = e % NC, beta = col / k, i = col % k;
      Pc[c * NC + col] = A.P[((2 * j + beta) * k + i) * int64_t(A.nr) + int64_t(c) * A.nb + l];
    }
    // T[row][col] = sum over the selected links Y (incl. X for part 0) of
    //               sum_c' Y[row][beta*h + c'] P(y)[beta*h + c'][col]
    for (int e = threadIdx.x; e < N * NC; e += blockDim.x) {
      const int row = e / NC, col = e % NC, beta = col / k, i = col % k;
      double2 t = make_double2(0, 0);
      for (int nbi = 0; nbi < 9; ++nbi) {
        int64_t y;
        if (nbi == 0) {
          if (part != 0) continue;
          y = x;
        } else {
          y = A.nbr[int64_t(nbi - 1) * A.V + x];
          const bool inside = (y / A.nb) == j;
          if (part == 0 ? !inside : (nbi != 1 + 2 * (part - 1) || inside)) continue;
        }
        const double2* Y = A.links + (x * 9 + nbi) * int64_t(N) * N;  // column-major
        const int64_t jy = y / A.nb, ly = y % A.nb;
        const double2* py = A.P + ((2 * jy + beta) * k + i) * int64_t(A.nr) + ly;
        for (int c = 0; c < h; ++c) cfma(t, Y[int64_t(beta * h + c) * N + row], py[int64_t(c) * A.nb]);
      }
      T[row * NC + col] = t;
    }
    __syncthreads();
#pragma unroll
    for (int xr = 0; xr < TI; ++xr) {
      const int r = rg * TI + xr;
      const int ar = r / k;
      for (int c = 0; c < h; ++c) {
        const double2 pr = Pc[c * NC + r];
#pragma unroll
        for (int yc = 0; yc < TI; ++yc) cfmac(acc[xr][yc], pr, T[(ar * h + c) * NC + cg * TI + yc]);
      }
    }
  }
  const int64_t jpos = A.pos_c ? A.pos_c[j] : j;
  const int nbidx = part == 0 ? 0 : 1 + 2 * (part - 1);
  double2* out = A.out + (jpos * 9 + nbidx) * int64_t(NC) * NC;
#pragma unroll
  for (int xr = 0; xr < TI; ++xr)
#pragma unroll
    for (int yc = 0; yc < TI; ++yc) {
      const int r = rg * TI + xr, c = cg * TI + yc;
      out[int64_t(c) * NC + r] = acc[xr][yc];
    }
}

}  // namespace

void galerkin_coarse(const GalerkinCoarseArgs& A, const int* nbr_c, int64_t Vc, hipStream_t st) {
  const int NC = 2 * A.k;
  CRK_REQUIRE(NC % 16 == 0 && NC <= 64, "2k must be 16, 32, 48 or 64");
  const dim3 g = dim3(unsigned(A.ncoarse * 5));
  const size_t lds = sizeof(double2) * size_t(A.N + A.N / 2) * NC;
  CRK_REQUIRE(lds <= 160 * 1024, "coarse Galerkin: LDS above 160 KiB");
  auto launch = [&](auto kern) {
    if (lds > 64 * 1024)
      CRK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  int(lds)));
    hipLaunchKernelGGL(kern, g, dim3(256), lds, st, A);
  };
  switch (NC / 16) {
    case 1: launch(galerkin_coarse_kernel<1>); break;
    case 2: launch(galerkin_coarse_kernel<2>); break;
    case 3: launch(galerkin_coarse_kernel<3>); break;
    default: launch(galerkin_coarse_kernel<4>); break;
  }
  CRK_LAUNCH_CHECK();
  hipLaunchKernelGGL(backward_links_kernel, dim3(unsigned(Vc * 4)), dim3(256), 0, st, A.out, nbr_c, Vc, NC, A.k);
  CRK_LAUNCH_CHECK();
}

}  // namespace crk
