// Batched chiral SVD truncation (paper, Sec. 3, Eqs. (5)-(6)).
//
// For every block Lambda_j and chirality alpha the N_r x m matrix
// A = Psi^(alpha)(Lambda_j) (normalised test vectors restricted to the block,
// components of one chirality) is factorised and its k dominant left singular
// vectors become the block of the prolongator P.
//
// Algorithm (one workgroup per (j, alpha), all in FP64):
//   1. G  = A^dag A                          (streamed from the test vectors)
//   2. G  = V diag(lambda) V^dag             (m <= 64: Householder tridiagonal
//                                             form + implicit QL; above: cyclic Jacobi)
//   3. B  = A V,  G2 = B^dag B               (B stored; G2 is nearly diagonal)
//   4. G2 = W diag(lambda2) W^dag            (Jacobi again, few sweeps)
//   5. U_k = B W_k diag(phase_i / sigma_i),  sigma_i = sqrt(lambda2_i)
// Step 1-2 alone lose accuracy for small sigma (the Gram matrix squares the
// condition number).  B's columns have norms sigma_i, so G2 carries errors of
// order eps*sigma_i*sigma_j and the second Jacobi resolves each pair to the
// accuracy of a one-sided Jacobi sweep; U_k = B W_k keeps orthogonality to
// working precision.  Phase: column i is multiplied by conj(s_i)/|s_i| with
// s_i the sum of the entries of the right singular vector (V W)_i.
//
// Row order inside a block on the device: rho = c'*|Lambda| + l (component c'
// of the chirality, local site l), which is contiguous in the field layouts.
#include <algorithm>

#include "field.h"
#include "kernels.h"
#include "svd.h"

namespace crk {

namespace {

constexpr int kThreads = 256;
constexpr int kBigMax = 128;  // largest m' (columns of a block matrix)

template <class T2>
__device__ __forceinline__ double2 ld2(const T2* p, int64_t i) {
  T2 v = p[i];
  return make_double2(double(v.x), double(v.y));
}

// Element e of rows [r0, r0+nrows) of the scaled block matrix: its value and
// its (row, column) in the chunk; consecutive e follow the source's memory order.
template <class T2>
__device__ __forceinline__ double2 block_row_elem(const ChiralSrc& src, const T2* base, const double* inv_norm,
                                                  int64_t j, int alpha, int r0, int nrows, int m, int e, int& rr,
                                                  int& i) {
  if (src.si == 1 && !src.aosoa) { i = e % m; rr = e / m; }  // columns contiguous in memory
  else { rr = e % nrows; i = e / nrows; }           // rows contiguous in memory
  const int rho = r0 + rr;
  const int c = rho / src.nb, l = rho % src.nb;
  const int64_t site = int64_t(j) * src.nb + l;
  const int64_t idx = src.aosoa ? aidx(i, alpha * src.h + c, site, src.Vp, src.ncomp)
                                : int64_t(i) * src.si + int64_t(alpha * src.h + c) * src.sc + site * src.ss;
  const double2 v = ld2(base, idx);
  const double s = inv_norm ? inv_norm[i] : 1.0;
  return make_double2(v.x * s, v.y * s);
}

// Load rows [r0, r0+nrows) of the scaled block matrix into lds[row][col] (ld = m).
template <class T2>
__device__ void load_block_rows(const ChiralSrc& src, const T2* base, const double* inv_norm, int64_t j, int alpha,
                                int r0, int nrows, int m, double2* lds, int ldm) {
  const int total = nrows * m;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int rr, i;
    const double2 v = block_row_elem(src, base, inv_norm, j, alpha, r0, nrows, m, e, rr, i);
    lds[rr * ldm + i] = v;
  }
}

// acc[x][y] += sum_rows conj(L[row][ti + GW x]) * L[row][tj + GW y] for
// y >= x: the columns of a thread's tile are GW apart, so the GW threads of a
// tile row read GW consecutive entries (no LDS bank conflicts).  The result is
// Hermitian: the entries with y < x lie below the diagonal and are the
// conjugates of entries another thread forms (gram_store writes both).  Each
// entry is summed over the rows in order.
template <int TI, int GW, int UNR = 1>
__device__ __forceinline__ void gram_accumulate(const double2* lds, int ldm, int nrows, int ti, int tj, int m,
                                                double2 (&acc)[TI][TI]) {
#pragma unroll UNR
  for (int r = 0; r < nrows; ++r) {
    double2 a[TI], b[TI];
#pragma unroll
    for (int x = 0; x < TI; ++x) {
      const int ia = ti + GW * x, ib = tj + GW * x;
      a[x] = ia < m ? lds[r * ldm + ia] : make_double2(0, 0);
      b[x] = ib < m ? lds[r * ldm + ib] : make_double2(0, 0);
    }
#pragma unroll
    for (int x = 0; x < TI; ++x)
#pragma unroll
      for (int y = x; y < TI; ++y) cfmac(acc[x][y], a[x], b[y]);
  }
}

// Stores the entries gram_accumulate formed and, above the diagonal blocks,
// their conjugates below it.
template <int TI, int GW>
__device__ __forceinline__ void gram_store(double2* G, int m, int ti, int tj, const double2 (&acc)[TI][TI]) {
#pragma unroll
  for (int x = 0; x < TI; ++x)
#pragma unroll
    for (int y = x; y < TI; ++y) {
      const int i = ti + GW * x, ii = tj + GW * y;
      if (i < m && ii < m) {
        G[i * m + ii] = acc[x][y];
        if (y > x) G[ii * m + i] = cconj(acc[x][y]);
      }
    }
}

constexpr int kChunk = 32;

// Rows [r0, r0+nrows) of a plain row-major matrix [N_r][m] (the rotated B = A V).
__device__ void load_plain_rows(const double2* Bp, int r0, int nrows, int m, double2* lds) {
  const int total = nrows * m;
  for (int e = threadIdx.x; e < total; e += blockDim.x) lds[e] = Bp[int64_t(r0) * m + e];
}

// G = A^dag A per (block, chirality): a GW x GW thread grid, each thread a
// TI x TI set of entries of G, rows and columns GW apart (GW = 16 for
// m <= 64, 32 for m <= 128).  PLAIN: A is a
// plain row-major [pair][N_r][m] matrix instead of the test vectors.
template <class T2, int TI, int GW, bool PLAIN>
__global__ __launch_bounds__(GW * GW) void gram_kernel(ChiralSrc src, const T2* __restrict__ base,
                                                       const double* __restrict__ inv_norm,
                                                       double2* __restrict__ G) {
  extern __shared__ double2 lds[];
  const int pair = blockIdx.x, alpha = pair & 1;
  const int64_t j = src.j0 + (pair >> 1);
  const int m = src.m, nr = src.h * src.nb;
  const int ti = threadIdx.x / GW, tj = threadIdx.x % GW;
  double2 acc[TI][TI];
#pragma unroll
  for (int x = 0; x < TI; ++x)
#pragma unroll
    for (int y = 0; y < TI; ++y) acc[x][y] = make_double2(0, 0);
  for (int r0 = 0; r0 < nr; r0 += kChunk) {
    const int nrows = min(kChunk, nr - r0);
    __syncthreads();
    if constexpr (PLAIN) load_plain_rows(reinterpret_cast<const double2*>(base) + int64_t(pair) * nr * m, r0, nrows, m, lds);
    else load_block_rows(src, base, inv_norm, j, alpha, r0, nrows, m, lds, m);
    __syncthreads();
    gram_accumulate<TI, GW>(lds, m, nrows, ti, tj, m, acc);
  }
  gram_store<TI, GW>(G + int64_t(pair) * m * m, m, ti, tj, acc);
}

// ---------------------------------------------------------------- Jacobi
// Hermitian eigendecomposition of a batch of m x m matrices (m <= 64), one
// workgroup each, matrix and eigenvectors in LDS.  Round-robin ordering: in
// each of mm-1 rounds the mm/2 disjoint pairs are rotated together.
struct Rot { double c, s; double2 e; };  // J = [[c, s], [-s e, c e]],  e = conj(g)/|g|

__device__ __forceinline__ void pair_of(int round, int k, int mm, int& p, int& q) {
  const int n = mm - 1;
  if (k == 0) { p = n; q = round; }
  else { p = (round + k) % n; q = (round - k + n) % n; }
  if (p > q) { int t = p; p = q; q = t; }
}

constexpr int kJacobiThreads = 1024;  // at most one 2x2 block update per thread (m' = 64: 32 x 32 pairs)
// Threads of a Jacobi workgroup: one per 2x2 block of a round (np^2, np = mm/2
// pairs), in whole wavefronts, at least 64 and at most kJacobiThreads.
inline int jacobi_threads(int m) {
  const int np = (m + (m & 1)) / 2;
  const int t = (np * np + 63) / 64 * 64;
  return t < 64 ? 64 : t > kJacobiThreads ? kJacobiThreads : t;
}

__global__ __launch_bounds__(kJacobiThreads) void jacobi_kernel(const double2* __restrict__ Gin, double* __restrict__ lam,
                                                          double2* __restrict__ Vout, int m, int max_sweeps,
                                                          double tol, int* __restrict__ sweeps_out) {
  extern __shared__ double2 sh[];
  const int mm = m + (m & 1);
  const int ld = mm + 1;  // padding against bank conflicts
  double2* G = sh;
  double2* V = sh + mm * ld;
  Rot* rot = reinterpret_cast<Rot*>(V + mm * ld);
  int* prs = reinterpret_cast<int*>(rot + mm / 2);
  __shared__ int n_rot;
  const int64_t b = blockIdx.x;
  const double2* Gb = Gin + b * m * m;
  for (int e = threadIdx.x; e < mm * mm; e += blockDim.x) {
    const int r = e / mm, c = e % mm;
    G[r * ld + c] = (r < m && c < m) ? Gb[r * m + c] : make_double2(0, 0);
    V[r * ld + c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) n_rot = 0;
    __syncthreads();
    for (int round = 0; round < mm - 1; ++round) {
      if (threadIdx.x < mm / 2) {
        int p, q;
        pair_of(round, threadIdx.x, mm, p, q);
        prs[2 * threadIdx.x] = p;
        prs[2 * threadIdx.x + 1] = q;
        const double a = G[p * ld + p].x, d = G[q * ld + q].x;
        const double2 g = G[p * ld + q];
        const double ag = hypot(g.x, g.y);
        Rot R{1.0, 0.0, make_double2(1.0, 0.0)};
        if (ag > tol * sqrt(fabs(a * d)) && ag > 0.0) {
          const double zeta = (d - a) / (2.0 * ag);
          const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          R.c = c;
          R.s = t * c;
          R.e = make_double2(g.x / ag, -g.y / ag);
          atomicAdd(&n_rot, 1);
        }
        rot[threadIdx.x] = R;
      }
      __syncthreads();
      // G <- J^dag G J on 2x2 blocks (pair a rows, pair b columns)
      const int np = mm / 2;
      for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
        const int ia = e / np, ib = e % np;
        const Rot Ra = rot[ia], Rb = rot[ib];
        const int pa = prs[2 * ia], qa = prs[2 * ia + 1], pb = prs[2 * ib], qb = prs[2 * ib + 1];
        const double2 m00 = G[pa * ld + pb], m01 = G[pa * ld + qb], m10 = G[qa * ld + pb], m11 = G[qa * ld + qb];
        // right multiply by Jb: col p' = c*col_p - s e col_q ; col q' = s col_p + c e col_q
        const double2 eb = Rb.e;
        const double2 se_b = make_double2(Rb.s * eb.x, Rb.s * eb.y), ce_b = make_double2(Rb.c * eb.x, Rb.c * eb.y);
        double2 t00 = cscale(m00, Rb.c) - cmul(m01, se_b);
        double2 t01 = cscale(m00, Rb.s) + cmul(m01, ce_b);
        double2 t10 = cscale(m10, Rb.c) - cmul(m11, se_b);
        double2 t11 = cscale(m10, Rb.s) + cmul(m11, ce_b);
        // left multiply by Ja^dag: row p' = c row_p - s conj(e) row_q ; row q' = s row_p + c conj(e) row_q
        const double2 ea = cconj(Ra.e);
        const double2 se_a = make_double2(Ra.s * ea.x, Ra.s * ea.y), ce_a = make_double2(Ra.c * ea.x, Ra.c * ea.y);
        G[pa * ld + pb] = cscale(t00, Ra.c) - cmul(se_a, t10);
        G[pa * ld + qb] = cscale(t01, Ra.c) - cmul(se_a, t11);
        G[qa * ld + pb] = cscale(t00, Ra.s) + cmul(ce_a, t10);
        G[qa * ld + qb] = cscale(t01, Ra.s) + cmul(ce_a, t11);
      }
      // V <- V J
      for (int e = threadIdx.x; e < mm * np; e += blockDim.x) {
        const int x = e / np, ib = e % np;
        const Rot Rb = rot[ib];
        const int pb = prs[2 * ib], qb = prs[2 * ib + 1];
        const double2 vp = V[x * ld + pb], vq = V[x * ld + qb];
        const double2 se = make_double2(Rb.s * Rb.e.x, Rb.s * Rb.e.y), ce = make_double2(Rb.c * Rb.e.x, Rb.c * Rb.e.y);
        V[x * ld + pb] = cscale(vp, Rb.c) - cmul(vq, se);
        V[x * ld + qb] = cscale(vp, Rb.s) + cmul(vq, ce);
      }
      __syncthreads();
    }
    const bool done = n_rot == 0;
    __syncthreads();
    if (done) break;
  }
  // Sort eigenvalues descending (ties by index) and write permuted columns.
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const double li = G[i * ld + i].x;
    int rank = 0;
    for (int jj = 0; jj < m; ++jj) {
      const double lj = G[jj * ld + jj].x;
      rank += (lj > li) || (lj == li && jj < i);
    }
    lam[b * m + rank] = li;
    for (int x = 0; x < m; ++x) Vout[b * m * m + int64_t(x) * m + rank] = V[x * ld + i];
  }
  if (threadIdx.x == 0 && sweeps_out) sweeps_out[b] = sweep;
}

// ---------------------------------------------------------------- first pass: tridiagonal QL
// Hermitian eigendecomposition G = V diag(lambda) V^dag of the first pass
// (m <= 64), one workgroup of kThreads per matrix:
//   1. Householder reduction G = Q T Q^dag with T Hermitian tridiagonal;
//      reflector k = I - tau u u^dag maps column k below the diagonal onto its
//      first entry alpha_k = T[k+1][k] (|alpha_k| = the column's norm), and u is
//      kept in that column;
//   2. Q = H_0 H_1 ... formed in place from the reflectors, last one first;
//   3. T = D S D^dag, S real symmetric with off-diagonal |alpha_k|, D the
//      diagonal of phases phi_{k+1} = phi_k alpha_k / |alpha_k|;
//   4. S = Z diag(lambda) Z^T by the implicit QL method with Wilkinson shifts
//      (the tql2 procedure of Bowdler, Martin, Reinsch and Wilkinson), the
//      rotations applied to the columns of Q D, so V = Q D Z.  One wavefront,
//      lane r holding row r of Q D's active columns; d and e live one entry per
//      lane and the scalar recurrences read and write them lane by lane;
//   5. eigenvalues descending, vectors permuted as jacobi_kernel writes them.
// An order of magnitude fewer flops than cyclic Jacobi; its vectors have the
// absolute accuracy of a backward-stable method, and the second pass (Jacobi
// on B^dag B) resolves the small singular values to working accuracy.
__device__ __forceinline__ double lane_get(double v, int lane) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(b)), lane));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(b >> 32)), lane));
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}
__device__ __forceinline__ double lane_set(double v, double x, int lane) {
  return int(threadIdx.x & 63) == lane ? x : v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

constexpr int kQlMaxIter = 60;  // QL iterations per eigenvalue before giving up (never reached in practice)

__global__ __launch_bounds__(kThreads) void heig_kernel(const double2* __restrict__ Gin, double* __restrict__ lam,
                                                        double2* __restrict__ Vout, int m, int* __restrict__ iters_out) {
  extern __shared__ double2 sh[];
  __shared__ double2 uv[64], pv[64], ev[64], ph[64];
  __shared__ double dv[64], er[64], tv[64];
  const int ld = m + 1;
  double2* A = sh;  // [m][ld]
  const int64_t b = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const double2* Gb = Gin + b * m * m;
  for (int e = t; e < m * m; e += blockDim.x) A[(e / m) * ld + e % m] = Gb[e];
  __syncthreads();
  // 1. reduction to tridiagonal form
  for (int k = 0; k + 2 < m; ++k) {
    const int n = m - 1 - k;  // trailing rows / columns k+1 .. m-1
    if (wid == 0) {
      const double2 x = lane < n ? A[(k + 1 + lane) * ld + k] : make_double2(0, 0);
      const double nx2 = wave_sum(x.x * x.x + x.y * x.y);
      const double2 x0 = make_double2(__shfl(x.x, 0), __shfl(x.y, 0));
      const double nx = sqrt(nx2), a0 = hypot(x0.x, x0.y);
      const double2 phs = a0 > 0.0 ? make_double2(x0.x / a0, x0.y / a0) : make_double2(1.0, 0.0);
      const double2 alpha = make_double2(-phs.x * nx, -phs.y * nx);
      double2 u = x;
      if (lane == 0) u = make_double2(x.x - alpha.x, x.y - alpha.y);
      const double un2 = wave_sum(u.x * u.x + u.y * u.y);
      const double tau = (nx2 > 0.0 && un2 > 0.0) ? 2.0 / un2 : 0.0;
      if (lane < n) {
        uv[lane] = u;
        A[(k + 1 + lane) * ld + k] = u;  // kept for forming Q
      }
      if (lane == 0) {
        tv[k] = tau;
        const bool nz = nx2 > 0.0;
        ev[k] = make_double2(nz ? alpha.x : x0.x, nz ? alpha.y : x0.y);  // T[k+1][k]
      }
    }
    __syncthreads();
    const double tau = tv[k];
    if (tau != 0.0) {
      // p = tau S u, S = A[k+1.., k+1..]: four threads per row
      {
        const int i = t >> 2, q = t & 3;
        double2 acc = make_double2(0, 0);
        if (i < n)
          for (int j = q; j < n; j += 4) cfma(acc, A[(k + 1 + i) * ld + k + 1 + j], uv[j]);
        acc.x += __shfl_xor(acc.x, 1);
        acc.y += __shfl_xor(acc.y, 1);
        acc.x += __shfl_xor(acc.x, 2);
        acc.y += __shfl_xor(acc.y, 2);
        if (q == 0 && i < n) pv[i] = make_double2(tau * acc.x, tau * acc.y);
      }
      __syncthreads();
      // w = p - (tau/2)(u^dag p) u
      if (wid == 0) {
        const double2 u = lane < n ? uv[lane] : make_double2(0, 0);
        const double2 pp = lane < n ? pv[lane] : make_double2(0, 0);
        double2 c = make_double2(0, 0);
        cfmac(c, u, pp);
        const double2 K = make_double2(0.5 * tau * wave_sum(c.x), 0.5 * tau * wave_sum(c.y));
        if (lane < n) pv[lane] = pp - cmul(K, u);
      }
      __syncthreads();
      // S -= u w^dag + w u^dag
      for (int e = t; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        const double2 ui = uv[i], uj = uv[j], wi = pv[i], wj = pv[j];
        double2& sij = A[(k + 1 + i) * ld + k + 1 + j];
        sij = sij - cmul(ui, cconj(wj)) - cmul(wi, cconj(uj));
      }
    }
    __syncthreads();
  }
  for (int i = t; i < m; i += blockDim.x) dv[i] = A[i * ld + i].x;
  if (t == 0 && m >= 2) ev[m - 2] = A[(m - 1) * ld + m - 2];
  __syncthreads();
  // 2. Q in place, last reflector first
  for (int e = t; e < 4; e += blockDim.x) {
    const int r = m - 2 + (e >> 1), c = m - 2 + (e & 1);
    if (r >= 0 && c >= 0) A[r * ld + c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int k = m - 3; k >= 0; --k) {
    const int n = m - 1 - k;
    // Q so far is the identity on index k+1
    for (int e = t; e < n; e += blockDim.x) {
      A[(k + 1 + e) * ld + k + 1] = make_double2(e == 0 ? 1.0 : 0.0, 0.0);
      if (e > 0) A[(k + 1) * ld + k + 1 + e] = make_double2(0, 0);
    }
    __syncthreads();
    const double tau = tv[k];
    if (tau != 0.0) {
      // y_c = tau sum_r conj(u_r) Q[r][c]
      {
        const int c = t >> 2, q = t & 3;
        double2 acc = make_double2(0, 0);
        if (c < n)
          for (int r = q; r < n; r += 4) cfmac(acc, A[(k + 1 + r) * ld + k], A[(k + 1 + r) * ld + k + 1 + c]);
        acc.x += __shfl_xor(acc.x, 1);
        acc.y += __shfl_xor(acc.y, 1);
        acc.x += __shfl_xor(acc.x, 2);
        acc.y += __shfl_xor(acc.y, 2);
        if (q == 0 && c < n) pv[c] = make_double2(tau * acc.x, tau * acc.y);
      }
      __syncthreads();
      for (int e = t; e < n * n; e += blockDim.x) {
        const int r = e / n, c = e % n;
        double2& qrc = A[(k + 1 + r) * ld + k + 1 + c];
        qrc = qrc - cmul(A[(k + 1 + r) * ld + k], pv[c]);
      }
    }
    __syncthreads();
  }
  for (int e = t; e < m; e += blockDim.x) {
    A[e] = make_double2(e == 0 ? 1.0 : 0.0, 0.0);       // row 0
    if (e > 0) A[e * ld] = make_double2(0, 0);         // column 0
  }
  // 3. phases
  if (t == 0) {
    double2 phi = make_double2(1.0, 0.0);
    ph[0] = phi;
    for (int j = 0; j + 1 < m; ++j) {
      const double2 a = ev[j];
      const double aa = hypot(a.x, a.y);
      er[j] = aa;
      if (aa > 0.0) phi = cmul(phi, make_double2(a.x / aa, a.y / aa));
      ph[j + 1] = phi;
    }
  }
  __syncthreads();
  for (int e = t; e < m * m; e += blockDim.x) {
    const int r = e / m, c = e % m;
    A[r * ld + c] = cmul(A[r * ld + c], ph[c]);
  }
  __syncthreads();
  // 4. implicit QL on (d, |alpha|), rotations applied to the columns of Q D
  if (wid == 0) {
    const double eps = 2.220446049250313e-16;
    double dd = lane < m ? dv[lane] : 0.0;
    double ee = lane + 1 < m ? er[lane] : 0.0;
    const bool row = lane < m;
    int its_total = 0;
    for (int l = 0; l < m; ++l) {
      int its = 0;
      while (true) {
        const double dn = __shfl_down(dd, 1);
        const bool small = lane >= l && (lane == m - 1 || fabs(ee) <= eps * (fabs(dd) + fabs(dn)));
        const uint64_t mask = __ballot(small);
        const int mm = int(__builtin_ctzll(mask));
        if (mm == l || its >= kQlMaxIter) break;
        ++its;
        const double dl = lane_get(dd, l), dl1 = lane_get(dd, l + 1), el = lane_get(ee, l), dm = lane_get(dd, mm);
        double g = (dl1 - dl) / (2.0 * el);
        double r = sqrt(g * g + 1.0);
        g = dm - dl + el / (g + (g >= 0.0 ? r : -r));
        double s = 1.0, c = 1.0, p = 0.0;
        bool deflated = false;
        double2 zc = row ? A[lane * ld + mm] : make_double2(0, 0);
        int i = mm - 1;
        for (; i >= l; --i) {
          const double ei = lane_get(ee, i);
          const double f = s * ei, bb = c * ei;
          r = sqrt(f * f + g * g);
          ee = lane_set(ee, r, i + 1);
          if (r == 0.0) {  // the recurrence split: d[i+1] -= p, e[mm] = 0, test again
            dd = lane_set(dd, lane_get(dd, i + 1) - p, i + 1);
            ee = lane_set(ee, 0.0, mm);
            deflated = true;
            break;
          }
          const double inv = 1.0 / r;
          s = f * inv;
          c = g * inv;
          g = lane_get(dd, i + 1) - p;
          r = (lane_get(dd, i) - g) * s + 2.0 * c * bb;
          p = s * r;
          dd = lane_set(dd, g + p, i + 1);
          g = c * r - bb;
          // columns i, i+1: z_{i+1} <- s z_i + c z_{i+1}, z_i <- c z_i - s z_{i+1}
          if (row) {
            const double2 zi = A[lane * ld + i];
            A[lane * ld + i + 1] = make_double2(s * zi.x + c * zc.x, s * zi.y + c * zc.y);
            zc = make_double2(c * zi.x - s * zc.x, c * zi.y - s * zc.y);
          }
        }
        if (row) A[lane * ld + (deflated ? i + 1 : l)] = zc;
        if (deflated) continue;
        dd = lane_set(dd, lane_get(dd, l) - p, l);
        ee = lane_set(ee, g, l);
        ee = lane_set(ee, 0.0, mm);
      }
      its_total += its;
    }
    if (row) dv[lane] = dd;
    if (lane == 0 && iters_out) iters_out[b] = its_total;
  }
  __syncthreads();
  // 5. descending order (ties by index), vectors permuted
  for (int i = t; i < m; i += blockDim.x) {
    const double li = dv[i];
    int rank = 0;
    for (int jj = 0; jj < m; ++jj) {
      const double lj = dv[jj];
      rank += (lj > li) || (lj == li && jj < i);
    }
    lam[b * m + rank] = li;
    for (int x = 0; x < m; ++x) Vout[b * m * m + int64_t(x) * m + rank] = A[x * ld + i];
  }
}

// ---------------------------------------------------------------- B = A V, G2 = B^dag B
constexpr int kRotChunk = 16;
static_assert(kThreads == 256 && kRotChunk == 16, "rotate_kernel: 8 row pairs x 32 column pairs of threads");

template <class T2, int TI>
__global__ __launch_bounds__(kThreads) void rotate_kernel(ChiralSrc src, const T2* __restrict__ base,
                                                          const double* __restrict__ inv_norm,
                                                          const double2* __restrict__ Vin, double2* __restrict__ B,
                                                          double2* __restrict__ G2) {
  extern __shared__ double2 lds[];
  const int m = src.m, nr = src.h * src.nb;
  const int pair = blockIdx.x, alpha = pair & 1;
  const int64_t j = src.j0 + (pair >> 1);
  const int la = m + 1;                // padded row stride of As: its rows sit in different LDS banks
  double2* Vs = lds;                   // [m][m]
  double2* As = Vs + m * m;            // [kRotChunk][m + 1]
  double2* Bs = As + kRotChunk * la;   // [kRotChunk][m]
  const double2* Vb = Vin + int64_t(pair) * m * m;
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) Vs[e] = Vb[e];
  const int ti = threadIdx.x / 16, tj = threadIdx.x % 16;
  double2 acc[TI][TI];
#pragma unroll
  for (int x = 0; x < TI; ++x)
#pragma unroll
    for (int y = 0; y < TI; ++y) acc[x][y] = make_double2(0, 0);
  double2* Bp = B + int64_t(pair) * nr * m;
  // the next chunk of A is loaded into registers while the current one is used
  constexpr int kPre = kRotChunk * 64 / kThreads;  // m <= 64
  double2 pre[kPre];
  int prr[kPre], pi[kPre];
#pragma unroll
  for (int u = 0; u < kPre; ++u) {
    const int e = threadIdx.x + u * kThreads, nrows0 = min(kRotChunk, nr);
    prr[u] = -1;
    if (e < nrows0 * m) pre[u] = block_row_elem(src, base, inv_norm, j, alpha, 0, nrows0, m, e, prr[u], pi[u]);
  }
  for (int r0 = 0; r0 < nr; r0 += kRotChunk) {
    const int nrows = min(kRotChunk, nr - r0);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPre; ++u)
      if (prr[u] >= 0) As[prr[u] * la + pi[u]] = pre[u];
    __syncthreads();
    if (r0 + kRotChunk < nr) {
      const int r1 = r0 + kRotChunk, nrows1 = min(kRotChunk, nr - r1);
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        const int e = threadIdx.x + u * kThreads;
        prr[u] = -1;
        if (e < nrows1 * m) pre[u] = block_row_elem(src, base, inv_norm, j, alpha, r1, nrows1, m, e, prr[u], pi[u]);
      }
    }
    {
      // thread (g, c) forms the 2 x 2 tile of B rows {g, g + 8} x columns
      // {c, c + 32}: every A and V value it reads from LDS feeds two products.
      // Each entry is summed over i in order, as a plain row-column product.
      const int c = threadIdx.x & 31, g = threadIdx.x >> 5;
      const int ra = g, rb = g + 8, ca = c, cb = c + 32;
      const int ra_ = ra < nrows ? ra : 0, rb_ = rb < nrows ? rb : 0;  // past the end: row/column 0, not stored
      const int ca_ = ca < m ? ca : 0, cb_ = cb < m ? cb : 0;
      double2 taa = make_double2(0, 0), tab = taa, tba = taa, tbb = taa;
#pragma unroll 4
      for (int i = 0; i < m; ++i) {
        const double2 xa = As[ra_ * la + i], xb = As[rb_ * la + i];
        const double2 va = Vs[i * m + ca_], vb = Vs[i * m + cb_];
        cfma(taa, xa, va);
        cfma(tab, xa, vb);
        cfma(tba, xb, va);
        cfma(tbb, xb, vb);
      }
      if (ra < nrows && ca < m) { Bs[ra * m + ca] = taa; Bp[int64_t(r0 + ra) * m + ca] = taa; }
      if (ra < nrows && cb < m) { Bs[ra * m + cb] = tab; Bp[int64_t(r0 + ra) * m + cb] = tab; }
      if (rb < nrows && ca < m) { Bs[rb * m + ca] = tba; Bp[int64_t(r0 + rb) * m + ca] = tba; }
      if (rb < nrows && cb < m) { Bs[rb * m + cb] = tbb; Bp[int64_t(r0 + rb) * m + cb] = tbb; }
    }
    __syncthreads();
    gram_accumulate<TI, 16, 4>(Bs, m, nrows, ti, tj, m, acc);
  }
  gram_store<TI, 16>(G2 + int64_t(pair) * m * m, m, ti, tj, acc);
}

// ---------------------------------------------------------------- U_k = B T
constexpr int kFinChunk = 32;

__global__ __launch_bounds__(kThreads) void finalize_kernel(int m, int nr, int k, const double2* __restrict__ Vin,
                                                            const double2* __restrict__ Win,
                                                            const double* __restrict__ lam2,
                                                            const double2* __restrict__ B, double2* __restrict__ P,
                                                            double* __restrict__ sigma, int nsig) {
  extern __shared__ double2 lds[];
  const int pair = blockIdx.x;
  double2* T = lds;             // [m][k]
  double2* Bs = T + m * k;      // [kFinChunk][m + 1]
  __shared__ double2 phase[64];
  __shared__ double sig[64];
  __shared__ double2 colsum[kBigMax];
  const double2* Vb = Vin + int64_t(pair) * m * m;
  const double2* Wb = Win + int64_t(pair) * m * m;
  // s_i = sum_x (V W)[x][i] = sum_y (sum_x V[x][y]) W[y][i]
  if (threadIdx.x < m) {
    double2 cs = make_double2(0, 0);
    for (int x = 0; x < m; ++x) cs = cs + Vb[int64_t(x) * m + threadIdx.x];
    colsum[threadIdx.x] = cs;
  }
  __syncthreads();
  if (threadIdx.x < k) {
    const int i = threadIdx.x;
    double2 s = make_double2(0, 0);
    for (int y = 0; y < m; ++y) cfma(s, colsum[y], Wb[int64_t(y) * m + i]);
    const double a = hypot(s.x, s.y);
    phase[i] = a > 0 ? make_double2(s.x / a, -s.y / a) : make_double2(1, 0);
    const double l = lam2[int64_t(pair) * m + i];
    sig[i] = l > 0 ? sqrt(l) : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < m * k; e += blockDim.x) {
    const int y = e / k, i = e % k;
    const double inv = sig[i] > 0 ? 1.0 / sig[i] : 0.0;
    const double2 w = cmul(Wb[int64_t(y) * m + i], phase[i]);
    T[y * k + i] = make_double2(w.x * inv, w.y * inv);
  }
  for (int i = threadIdx.x; i < nsig; i += blockDim.x) {
    const double l = lam2[int64_t(pair) * m + i];
    sigma[int64_t(pair) * nsig + i] = l > 0 ? sqrt(l) : 0.0;
  }
  const double2* Bp = B + int64_t(pair) * nr * m;
  double2* Pp = P + int64_t(pair) * k * nr;
  const int mp = m + 1;  // padded row stride: lanes of consecutive rows hit different LDS banks
  for (int r0 = 0; r0 < nr; r0 += kFinChunk) {
    const int nrows = min(kFinChunk, nr - r0);
    __syncthreads();
    for (int e = threadIdx.x; e < nrows * m; e += blockDim.x) Bs[(e / m) * mp + e % m] = Bp[int64_t(r0) * m + e];
    __syncthreads();
    for (int e = threadIdx.x; e < nrows * k; e += blockDim.x) {
      const int i = e / nrows, rr = e % nrows;
      double2 t = make_double2(0, 0);
#pragma unroll 8
      for (int y = 0; y < m; ++y) cfma(t, Bs[rr * mp + y], T[y * k + i]);
      Pp[int64_t(i) * nr + r0 + rr] = t;
    }
  }
}

// ---------------------------------------------------------------- m' in (64, 128]
// The m x m Gram matrix and its eigenvectors no longer fit in LDS together
// (2 x 264 KiB at m = 128), so the eigendecomposition is split:
//   * jacobi_seg_kernel keeps G in LDS as a packed Hermitian upper triangle
//     (132 KiB at m = 128), runs up to kSegSweeps sweeps of the same cyclic
//     round-robin Jacobi as jacobi_kernel, records every round's rotations in
//     global memory and writes G back (packed) for the next segment;
//   * replay_kernel applies the recorded rotations to V (global, mm x mm):
//     one wavefront per row of V, the row staged in LDS, lane k rotating the
//     columns of pair k in every round (the rounds of a row run in order within
//     the wavefront; the pairs of one round are disjoint);
//   * jacobi_sort_kernel orders the eigenvalues descending and writes the
//     permuted eigenvectors in the layout jacobi_kernel writes.
// The segments repeat until a sweep makes no rotation (or the sweep limit):
// the result equals that of one Jacobi over all sweeps.
constexpr int kBigThreads = 1024;
constexpr int kSegSweeps = 4;
constexpr int kReplayRounds = 32;  // rounds of rotations staged in LDS per chunk

struct RotRec { double c, s, ex, ey; };

__device__ __forceinline__ int tri_idx(int i, int j, int n) {  // i <= j, packed upper triangle of n x n
  return i * (2 * n - i + 1) / 2 + (j - i);
}
__device__ __forceinline__ double2 tri_get(const double2* T, int i, int j, int n) {
  return i <= j ? T[tri_idx(i, j, n)] : cconj(T[tri_idx(j, i, n)]);
}
__device__ __forceinline__ void tri_set(double2* T, int i, int j, int n, double2 v) {
  if (i <= j) T[tri_idx(i, j, n)] = v;
  else T[tri_idx(j, i, n)] = cconj(v);
}

// state[3*b]: 1 once converged; state[3*b+1]: rounds recorded by the last
// segment; state[3*b+2]: sweeps done so far.
__global__ __launch_bounds__(kBigThreads) void jacobi_seg_kernel(const double2* __restrict__ Gin,
                                                                 double2* __restrict__ Gp, RotRec* __restrict__ rec,
                                                                 int* __restrict__ state, int m, int first,
                                                                 int max_sweeps, double tol) {
  extern __shared__ double2 sh[];
  const int mm = m + (m & 1), np = mm / 2, ntri = mm * (mm + 1) / 2;
  double2* T = sh;
  Rot* rot = reinterpret_cast<Rot*>(T + ntri);
  int* prs = reinterpret_cast<int*>(rot + np);
  __shared__ int n_rot;
  const int64_t b = blockIdx.x;
  int* st = state + 3 * b;
  if (!first && (st[0] || st[2] >= max_sweeps)) {
    if (threadIdx.x == 0) st[1] = 0;
    return;
  }
  double2* Gpb = Gp + b * ntri;
  if (first) {
    const double2* Gb = Gin + b * m * m;
    for (int e = threadIdx.x; e < mm * mm; e += blockDim.x) {
      const int r = e / mm, c = e % mm;
      if (r <= c) T[tri_idx(r, c, mm)] = (r < m && c < m) ? Gb[r * m + c] : make_double2(0, 0);
    }
  } else {
    for (int e = threadIdx.x; e < ntri; e += blockDim.x) T[e] = Gpb[e];
  }
  const int done0 = first ? 0 : st[2];
  RotRec* rb = rec + b * int64_t(kSegSweeps) * (mm - 1) * np;
  int sweep = 0;
  bool converged = false;
  for (; sweep < kSegSweeps && done0 + sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) n_rot = 0;
    __syncthreads();
    for (int round = 0; round < mm - 1; ++round) {
      if (threadIdx.x < np) {
        int p, q;
        pair_of(round, threadIdx.x, mm, p, q);
        prs[2 * threadIdx.x] = p;
        prs[2 * threadIdx.x + 1] = q;
        const double a = T[tri_idx(p, p, mm)].x, d = T[tri_idx(q, q, mm)].x;
        const double2 g = T[tri_idx(p, q, mm)];
        const double ag = hypot(g.x, g.y);
        Rot R{1.0, 0.0, make_double2(1.0, 0.0)};
        if (ag > tol * sqrt(fabs(a * d)) && ag > 0.0) {
          const double zeta = (d - a) / (2.0 * ag);
          const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          R.c = c;
          R.s = t * c;
          R.e = make_double2(g.x / ag, -g.y / ag);
          atomicAdd(&n_rot, 1);
        }
        rot[threadIdx.x] = R;
        rb[(int64_t(sweep) * (mm - 1) + round) * np + threadIdx.x] = RotRec{R.c, R.s, R.e.x, R.e.y};
      }
      __syncthreads();
      // G <- J^dag G J on the 2x2 blocks of pair a (rows) and pair b (columns),
      // each unordered block pair once; the block (b, a) is its conjugate transpose
      for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
        const int ia = e / np, ib = e % np;
        if (ia > ib) continue;
        const Rot Ra = rot[ia], Rb = rot[ib];
        const int pa = prs[2 * ia], qa = prs[2 * ia + 1], pb = prs[2 * ib], qb = prs[2 * ib + 1];
        const double2 m00 = tri_get(T, pa, pb, mm), m01 = tri_get(T, pa, qb, mm);
        const double2 m10 = tri_get(T, qa, pb, mm), m11 = tri_get(T, qa, qb, mm);
        const double2 eb = Rb.e;
        const double2 se_b = make_double2(Rb.s * eb.x, Rb.s * eb.y), ce_b = make_double2(Rb.c * eb.x, Rb.c * eb.y);
        double2 t00 = cscale(m00, Rb.c) - cmul(m01, se_b);
        double2 t01 = cscale(m00, Rb.s) + cmul(m01, ce_b);
        double2 t10 = cscale(m10, Rb.c) - cmul(m11, se_b);
        double2 t11 = cscale(m10, Rb.s) + cmul(m11, ce_b);
        const double2 ea = cconj(Ra.e);
        const double2 se_a = make_double2(Ra.s * ea.x, Ra.s * ea.y), ce_a = make_double2(Ra.c * ea.x, Ra.c * ea.y);
        const double2 n00 = cscale(t00, Ra.c) - cmul(se_a, t10);
        const double2 n01 = cscale(t01, Ra.c) - cmul(se_a, t11);
        const double2 n10 = cscale(t00, Ra.s) + cmul(ce_a, t10);
        const double2 n11 = cscale(t01, Ra.s) + cmul(ce_a, t11);
        tri_set(T, pa, pb, mm, n00);
        tri_set(T, pa, qb, mm, n01);
        if (ia != ib) tri_set(T, qa, pb, mm, n10);  // on the diagonal block it is conj(n01)
        tri_set(T, qa, qb, mm, n11);
      }
      __syncthreads();
    }
    const bool none = n_rot == 0;
    __syncthreads();
    if (none) { converged = true; break; }  // that sweep's rotations are all 1: not replayed
  }
  for (int e = threadIdx.x; e < ntri; e += blockDim.x) Gpb[e] = T[e];
  if (threadIdx.x == 0) {
    st[0] = converged ? 1 : 0;
    st[1] = sweep * (mm - 1);
    st[2] = done0 + sweep;
  }
}

// One wavefront per row x of V (mm x mm, global), kBigThreads / 64 rows per
// workgroup; the rows of matrix b are spread over ceil(mm / 16) workgroups.
__global__ __launch_bounds__(kBigThreads) void replay_kernel(double2* __restrict__ Vg, const RotRec* __restrict__ rec,
                                                             const int* __restrict__ state, int m, int first,
                                                             int wg_per_matrix) {
  __shared__ double2 row[kBigThreads / 64][kBigMax];
  __shared__ RotRec prm[kReplayRounds][kBigMax / 2];
  const int mm = m + (m & 1), np = mm / 2;
  const int64_t b = blockIdx.x / wg_per_matrix;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int x = (blockIdx.x % wg_per_matrix) * (kBigThreads / 64) + w;
  const int nrounds = state[3 * b + 1];
  double2* Vb = Vg + b * mm * mm;
  if (nrounds == 0 && !first) return;  // uniform over the workgroup
  const bool live = x < mm;
  if (live)  // the first segment starts from V = 1
    for (int c = lane; c < mm; c += 64)
      row[w][c] = first ? make_double2(x == c ? 1.0 : 0.0, 0.0) : Vb[int64_t(x) * mm + c];
  const RotRec* rb = rec + b * int64_t(kSegSweeps) * (mm - 1) * np;
  for (int t0 = 0; t0 < nrounds; t0 += kReplayRounds) {
    const int nr = min(kReplayRounds, nrounds - t0);
    __syncthreads();  // every wavefront is done with the previous chunk of parameters
    for (int e = threadIdx.x; e < nr * np; e += blockDim.x) prm[e / np][e % np] = rb[int64_t(t0) * np + e];
    __syncthreads();
    if (!live) continue;
    for (int t = 0; t < nr; ++t) {
      const int round = (t0 + t) % (mm - 1);
      if (lane < np) {
        int p, q;
        pair_of(round, lane, mm, p, q);
        const RotRec R = prm[t][lane];
        const double2 se = make_double2(R.s * R.ex, R.s * R.ey), ce = make_double2(R.c * R.ex, R.c * R.ey);
        const double2 vp = row[w][p], vq = row[w][q];
        row[w][p] = cscale(vp, R.c) - cmul(vq, se);
        row[w][q] = cscale(vp, R.s) + cmul(vq, ce);
      }
      // the next round reads columns other lanes of this wavefront wrote
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  if (live)
    for (int c = lane; c < mm; c += 64) Vb[int64_t(x) * mm + c] = row[w][c];
}

// Eigenvalues descending (ties by index) and the permuted eigenvectors, as jacobi_kernel writes them.
__global__ __launch_bounds__(kBigMax) void jacobi_sort_kernel(const double2* __restrict__ Gp,
                                                             const double2* __restrict__ Vg, double* __restrict__ lam,
                                                             double2* __restrict__ Vout, const int* __restrict__ state,
                                                             int* __restrict__ sweeps_out, int m) {
  const int mm = m + (m & 1), ntri = mm * (mm + 1) / 2;
  const int64_t b = blockIdx.x;
  const double2* T = Gp + b * ntri;
  const double2* Vb = Vg + b * mm * mm;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const double li = T[tri_idx(i, i, mm)].x;
    int rank = 0;
    for (int jj = 0; jj < m; ++jj) {
      const double lj = T[tri_idx(jj, jj, mm)].x;
      rank += (lj > li) || (lj == li && jj < i);
    }
    lam[b * m + rank] = li;
    for (int x = 0; x < m; ++x) Vout[b * m * m + int64_t(x) * m + rank] = Vb[int64_t(x) * mm + i];
  }
  if (threadIdx.x == 0 && sweeps_out) sweeps_out[b] = state[3 * b + 2];
}

// B = A V for m <= 128: kRotBigRows rows of A per pass in LDS, each thread one
// column c and kRotBigRows / 8 rows (V read from global, reused across them).
constexpr int kRotBigRows = 64;

template <class T2>
__global__ __launch_bounds__(kBigThreads) void rotate_big_kernel(ChiralSrc src, const T2* __restrict__ base,
                                                                 const double* __restrict__ inv_norm,
                                                                 const double2* __restrict__ Vin,
                                                                 double2* __restrict__ B) {
  extern __shared__ double2 lds[];  // [kRotBigRows][m]
  const int m = src.m, nr = src.h * src.nb;
  const int pair = blockIdx.x, alpha = pair & 1;
  const int64_t j = src.j0 + (pair >> 1);
  const double2* Vb = Vin + int64_t(pair) * m * m;
  double2* Bp = B + int64_t(pair) * nr * m;
  const int c = threadIdx.x % kBigMax, g = threadIdx.x / kBigMax;  // g in [0, 8)
  constexpr int kRows = kRotBigRows / (kBigThreads / kBigMax);
  for (int r0 = 0; r0 < nr; r0 += kRotBigRows) {
    const int nrows = min(kRotBigRows, nr - r0);
    __syncthreads();
    load_block_rows(src, base, inv_norm, j, alpha, r0, nrows, m, lds, m);
    __syncthreads();
    if (c >= m) continue;
    double2 acc[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u) acc[u] = make_double2(0, 0);
    for (int i = 0; i < m; ++i) {
      const double2 v = Vb[int64_t(i) * m + c];
#pragma unroll
      for (int u = 0; u < kRows; ++u) {
        const int rr = g + 8 * u;
        if (rr < nrows) cfma(acc[u], lds[rr * m + i], v);
      }
    }
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
      const int rr = g + 8 * u;
      if (rr < nrows) Bp[int64_t(r0 + rr) * m + c] = acc[u];
    }
  }
}

// Allow dynamic LDS beyond the 64 KiB default (gfx950 has 160 KiB per CU).
// Dynamic LDS above 64 KiB must be enabled per kernel (gfx950: 160 KiB per workgroup,
// static LDS included).
template <class K> void allow_lds(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return;
  CRK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(bytes)));
}

template <class T2, bool PLAIN>
void launch_gram(const ChiralSrc& s, const void* base, const double* inv_norm, double2* G, hipStream_t st) {
  const size_t lds = sizeof(double2) * kChunk * s.m;
  const dim3 grid = dim3(unsigned(2 * s.nblocks));
  const T2* b = static_cast<const T2*>(base);
  if (s.m <= 16) hipLaunchKernelGGL((gram_kernel<T2, 1, 16, PLAIN>), grid, dim3(256), lds, st, s, b, inv_norm, G);
  else if (s.m <= 32) hipLaunchKernelGGL((gram_kernel<T2, 2, 16, PLAIN>), grid, dim3(256), lds, st, s, b, inv_norm, G);
  else if (s.m <= 48) hipLaunchKernelGGL((gram_kernel<T2, 3, 16, PLAIN>), grid, dim3(256), lds, st, s, b, inv_norm, G);
  else if (s.m <= 64) hipLaunchKernelGGL((gram_kernel<T2, 4, 16, PLAIN>), grid, dim3(256), lds, st, s, b, inv_norm, G);
  else if (s.m <= 96) hipLaunchKernelGGL((gram_kernel<T2, 3, 32, PLAIN>), grid, dim3(1024), lds, st, s, b, inv_norm, G);
  else hipLaunchKernelGGL((gram_kernel<T2, 4, 32, PLAIN>), grid, dim3(1024), lds, st, s, b, inv_norm, G);
  CRK_LAUNCH_CHECK();
}

template <class T2>
void launch_rotate(const ChiralSrc& s, const void* base, const double* inv_norm, const double2* V, double2* B,
                   double2* G2, hipStream_t st) {
  const size_t lds = sizeof(double2) * (size_t(s.m) * s.m + kRotChunk * (2 * size_t(s.m) + 1));
  const dim3 grid = dim3(unsigned(2 * s.nblocks));
  const T2* b = static_cast<const T2*>(base);
  allow_lds(rotate_kernel<T2, 1>, lds); allow_lds(rotate_kernel<T2, 2>, lds);
  allow_lds(rotate_kernel<T2, 3>, lds); allow_lds(rotate_kernel<T2, 4>, lds);
  if (s.m <= 16) hipLaunchKernelGGL((rotate_kernel<T2, 1>), grid, dim3(kThreads), lds, st, s, b, inv_norm, V, B, G2);
  else if (s.m <= 32) hipLaunchKernelGGL((rotate_kernel<T2, 2>), grid, dim3(kThreads), lds, st, s, b, inv_norm, V, B, G2);
  else if (s.m <= 48) hipLaunchKernelGGL((rotate_kernel<T2, 3>), grid, dim3(kThreads), lds, st, s, b, inv_norm, V, B, G2);
  else hipLaunchKernelGGL((rotate_kernel<T2, 4>), grid, dim3(kThreads), lds, st, s, b, inv_norm, V, B, G2);
  CRK_LAUNCH_CHECK();
}

size_t heig_lds(int m) { return sizeof(double2) * size_t(m) * (m + 1); }

size_t jacobi_lds(int m) {
  const int mm = m + (m & 1), ld = mm + 1;
  return sizeof(double2) * 2 * mm * ld + sizeof(Rot) * (mm / 2) + sizeof(int) * mm;
}

}  // namespace

namespace {

// Eigendecomposition of the batch's m x m Hermitian matrices for 64 < m <= 128:
// Jacobi segments (G packed in LDS) alternating with the replay of their
// rotations onto V, then the sort.  Converged matrices skip the later segments.
void big_eig(const SvdWork& w, const double2* Gin, double* lam, double2* Vout, int* sweeps_out, int m, unsigned npair,
             double tol, hipStream_t st) {
  const int mm = m + (m & 1), ntri = mm * (mm + 1) / 2;
  const size_t lds = sizeof(double2) * ntri + sizeof(Rot) * (mm / 2) + sizeof(int) * mm;
  allow_lds(jacobi_seg_kernel, lds);
  const int wgpm = (mm + kBigThreads / 64 - 1) / (kBigThreads / 64);
  const int max_sweeps = 40;
  for (int seg = 0; seg * kSegSweeps < max_sweeps; ++seg) {
    hipLaunchKernelGGL(jacobi_seg_kernel, dim3(npair), dim3(kBigThreads), lds, st, Gin, w.Gp,
                       static_cast<RotRec*>(w.rec), w.state, m,
                       int(seg == 0), max_sweeps, tol);
    CRK_LAUNCH_CHECK();
    hipLaunchKernelGGL(replay_kernel, dim3(npair * unsigned(wgpm)), dim3(kBigThreads), 0, st, w.Vg,
                       static_cast<const RotRec*>(w.rec), w.state, m,
                       int(seg == 0), wgpm);
    CRK_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(jacobi_sort_kernel, dim3(npair), dim3(kBigMax), 0, st, w.Gp, w.Vg, lam, Vout, w.state,
                     sweeps_out, m);
  CRK_LAUNCH_CHECK();
}

}  // namespace

void chiral_svd(const ChiralSrc& s, int src_is_double, const void* base, const double* inv_norm, int k,
                const SvdWork& w, int64_t wcap, double2* P, double* sigma, hipStream_t st) {
  CRK_REQUIRE(s.m >= 1 && s.m <= kBigMax, "m' must be in [1, 128]");
  const int nr = s.h * s.nb;
  CRK_REQUIRE(k >= 1 && k <= s.m && k <= nr, "k must satisfy 1 <= k <= min(m', N_r)");
  CRK_REQUIRE(k <= 64, "k above 64 is not supported by the SVD finaliser");
  CRK_REQUIRE(wcap >= 1, "SVD work space must hold at least one block");
  const int m = s.m;
  const double tol = 1e-15;
  const int nsig = m < nr ? m : nr;
  const bool big = m > 64;
  const size_t lds = sizeof(double2) * (size_t(m) * k + size_t(kFinChunk) * (m + 1));
  CRK_REQUIRE(lds <= 160 * 1024, "SVD finaliser: m' * k too large for LDS");
  if (!big) {
    allow_lds(heig_kernel, heig_lds(m));
    allow_lds(jacobi_kernel, jacobi_lds(m));
  }
  allow_lds(finalize_kernel, lds);
  for (int64_t j0 = 0; j0 < s.nblocks; j0 += wcap) {
    ChiralSrc b = s;
    b.j0 = j0;
    b.nblocks = std::min(wcap, s.nblocks - j0);
    const unsigned npair = unsigned(2 * b.nblocks);
    if (src_is_double) launch_gram<double2, false>(b, base, inv_norm, w.G, st);
    else launch_gram<float2, false>(b, base, inv_norm, w.G, st);
    if (!big) {
      hipLaunchKernelGGL(heig_kernel, dim3(npair), dim3(kThreads), heig_lds(m), st, w.G, w.lam, w.V, m, w.sweeps);
      CRK_LAUNCH_CHECK();
      if (src_is_double) launch_rotate<double2>(b, base, inv_norm, w.V, w.B, w.G2, st);
      else launch_rotate<float2>(b, base, inv_norm, w.V, w.B, w.G2, st);
      hipLaunchKernelGGL(jacobi_kernel, dim3(npair), dim3(jacobi_threads(m)), jacobi_lds(m), st, w.G2, w.lam2, w.W, m,
                         40, tol, w.sweeps ? w.sweeps + npair : nullptr);
      CRK_LAUNCH_CHECK();
    } else {
      big_eig(w, w.G, w.lam, w.V, w.sweeps, m, npair, tol, st);
      const size_t rl = sizeof(double2) * kRotBigRows * m;
      if (src_is_double) {
        allow_lds(rotate_big_kernel<double2>, rl);
        hipLaunchKernelGGL(rotate_big_kernel<double2>, dim3(npair), dim3(kBigThreads), rl, st, b,
                           static_cast<const double2*>(base), inv_norm, w.V, w.B);
      } else {
        allow_lds(rotate_big_kernel<float2>, rl);
        hipLaunchKernelGGL(rotate_big_kernel<float2>, dim3(npair), dim3(kBigThreads), rl, st, b,
                           static_cast<const float2*>(base), inv_norm, w.V, w.B);
      }
      CRK_LAUNCH_CHECK();
      launch_gram<double2, true>(b, w.B, nullptr, w.G2, st);
      big_eig(w, w.G2, w.lam2, w.W, w.sweeps ? w.sweeps + npair : nullptr, m, npair, tol, st);
    }
    hipLaunchKernelGGL(finalize_kernel, dim3(npair), dim3(kThreads), lds, st, m, nr, k, w.V, w.W, w.lam2, w.B,
                       P + 2 * j0 * int64_t(k) * nr, sigma + 2 * j0 * int64_t(nsig), nsig);
    CRK_LAUNCH_CHECK();
  }
}

namespace {
size_t big_bytes_per_pair(int m) {
  if (m <= 64) return 0;
  const size_t mm = size_t(m + (m & 1)), ntri = mm * (mm + 1) / 2;
  return sizeof(double2) * (ntri + mm * mm) + sizeof(RotRec) * kSegSweeps * (mm - 1) * (mm / 2) + 3 * sizeof(int) +
         3 * 256;
}
}  // namespace

size_t svd_work_bytes(int m, int nr, int64_t nblocks) {
  const size_t np = size_t(2 * nblocks);
  return np * (sizeof(double2) * (4 * size_t(m) * m + size_t(nr) * m) + sizeof(double) * 2 * m + 2 * sizeof(int) +
               big_bytes_per_pair(m)) + 256 * 12;
}

SvdWork svd_work_carve(void* p, int m, int nr, int64_t nblocks) {
  const size_t np = size_t(2 * nblocks);
  char* c = static_cast<char*>(p);
  auto take = [&](size_t n) { char* r = c; c += (n + 255) & ~size_t(255); return r; };
  SvdWork w;
  w.G = reinterpret_cast<double2*>(take(sizeof(double2) * np * m * m));
  w.V = reinterpret_cast<double2*>(take(sizeof(double2) * np * m * m));
  w.G2 = reinterpret_cast<double2*>(take(sizeof(double2) * np * m * m));
  w.W = reinterpret_cast<double2*>(take(sizeof(double2) * np * m * m));
  w.B = reinterpret_cast<double2*>(take(sizeof(double2) * np * nr * m));
  w.lam = reinterpret_cast<double*>(take(sizeof(double) * np * m));
  w.lam2 = reinterpret_cast<double*>(take(sizeof(double) * np * m));
  w.sweeps = reinterpret_cast<int*>(take(sizeof(int) * 2 * np));
  w.Gp = nullptr;
  w.Vg = nullptr;
  w.rec = nullptr;
  w.state = nullptr;
  if (m > 64) {
    const size_t mm = size_t(m + (m & 1)), ntri = mm * (mm + 1) / 2;
    w.Gp = reinterpret_cast<double2*>(take(sizeof(double2) * np * ntri));
    w.Vg = reinterpret_cast<double2*>(take(sizeof(double2) * np * mm * mm));
    w.rec = take(sizeof(RotRec) * np * kSegSweeps * (mm - 1) * (mm / 2));
    w.state = reinterpret_cast<int*>(take(sizeof(int) * 3 * np));
  }
  return w;
}

}  // namespace crk
