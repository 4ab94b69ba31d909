// Selected eigenstates by block shift-invert (Appendix B, Eqs. (B1)-(B15)):
// the kernels of one iteration.  B = X^{-1} S C with X = alpha S - H factored
// by the upward sweep as X = L D L^T front by front (Eq. (B5)): each front f
// keeps A_f^{-1} (the inverse of its pivot block, the block of D) in the top
// J_f rows of its panel and L_f = B_f A_f^{-1} (U_f x J_f) in the L buffer.
// The product X^{-1} y takes the three steps of Eqs. (B8)-(B14):
//   forward  (B8)-(B9):  z_J = y_J - (updates of the children), and the
//                         front's update w_f = (children's updates on U_f)
//                         + L_f z_J, passed to the parent;
//   diagonal (B10)-(B11): z_J <- A_f^{-1} z_J;
//   backward (B12)-(B14): x_J = z_J - L_f^T x_U, root first.
// Block vectors hold EIG_NR = 16 columns; complex ones are row-major
// [row][column] in the permuted order of the dissection, real ones row-major
// in the caller's order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace ndrho {

// y[q][c] = sum_e A_ve x[col_e][c] with v = perm[q] (sparse A in CSR, real x
// in the caller's order, complex y in the permuted order): one thread per
// (q, c), columns fastest.
__global__ __launch_bounds__(256) void k_spmm_perm(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                   const double* __restrict__ a, const int32_t* __restrict__ perm,
                                                   int64_t n, const double* __restrict__ x, double2* __restrict__ y) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= n * EIG_NR) return;
  const int64_t q = t / EIG_NR;
  const int c = static_cast<int>(t % EIG_NR);
  const int64_t v = perm[q];
  double s = 0.0;
  for (int64_t e = rp[v]; e < rp[v + 1]; ++e) s += a[e] * x[int64_t(col[e]) * EIG_NR + c];
  y[t] = make_double2(s, 0.0);
}

// w[v][c] = sum_e A_ve x[col_e][c] for real x, w of NC columns (caller's order).
template <int NC>
__global__ __launch_bounds__(256) void k_spmm(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                              const double* __restrict__ a, int64_t n, const double* __restrict__ x,
                                              double* __restrict__ w) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= n * NC) return;
  const int64_t v = t / NC;
  const int c = static_cast<int>(t % NC);
  double s = 0.0;
  for (int64_t e = rp[v]; e < rp[v + 1]; ++e) s += a[e] * x[int64_t(col[e]) * NC + c];
  w[t] = s;
}

// Forward gather of one depth (Eq. (B8)): for every local row r of front f
// (pivot rows J, then update rows U), the sum over the children (in order)
// of their update entries that map onto r, through each child's inverse map
// (local row of the parent -> row of the child's update, or -1).  Pivot rows:
// z[j0 + r] = y[j0 + r] - sum; update rows: w_f[r - nj] = sum (the product
// L_f z_J is added by the grouped product that follows).  A tile covers
// EIG_GROWS rows x EIG_NR columns of one front.
__global__ __launch_bounds__(256) void k_solve_gather(const SolveFront* __restrict__ fronts,
                                                      const SolveChild* __restrict__ kids,
                                                      const int32_t* __restrict__ inv, const SolveTile* __restrict__ tiles,
                                                      const double2* __restrict__ y, double2* __restrict__ z,
                                                      double2* __restrict__ w) {
  const SolveTile tl = tiles[blockIdx.x];
  const SolveFront f = fronts[tl.front];
  const int r = tl.r0 + threadIdx.x / EIG_NR;
  const int c = threadIdx.x % EIG_NR;
  if (r >= f.nj + f.nu) return;
  double2 s = make_double2(0.0, 0.0);
  for (int k = 0; k < f.child_count; ++k) {
    const SolveChild ch = kids[f.child_begin + k];
    const int i = inv[ch.inv_off + r];
    if (i >= 0) {
      const double2 u = w[ch.w_off + int64_t(i) * EIG_NR + c];
      s.x += u.x;
      s.y += u.y;
    }
  }
  if (r < f.nj) {
    const int64_t g = (f.j0 + r) * EIG_NR + c;
    const double2 v = y[g];
    z[g] = make_double2(v.x - s.x, v.y - s.y);
  } else {
    w[f.w_off + int64_t(r - f.nj) * EIG_NR + c] = s;
  }
}

// Grouped tall-skinny complex product, one 64-row tile of one problem per
// workgroup: C[r][c] = (C0[r][c] if HAS_C0) + sign * sum_k op(A)[r][k] B[k][c],
// r < M, k < K, c < EIG_NR.  A is column-major (lda), op(A) = A or A^T (A^T:
// A is K x M); row k of B is b[b_off + k], or b[idx[b_off + k]] with GATHER.
// K is staged through LDS by 16.
constexpr int TS_BM = 64, TS_BK = 16;

template <bool TRANS, bool GATHER, bool HAS_C0, bool NEG>
__global__ __launch_bounds__(256) void k_tsgemm(const TsProb* __restrict__ probs, const TsTile* __restrict__ tiles,
                                                const double2* __restrict__ A, const double2* __restrict__ B,
                                                const int32_t* __restrict__ idx, const double2* C0,
                                                double2* C) {
  __shared__ double2 sa[TS_BK][TS_BM + 1];
  __shared__ double2 sb[TS_BK][EIG_NR];
  const TsTile tl = tiles[blockIdx.x];
  const TsProb p = probs[tl.prob];
  const int tid = threadIdx.x;
  const int row = tid % TS_BM, cg = tid / TS_BM;  // output row in the tile, column group of 4
  const int m0 = tl.m0;
  double2 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = make_double2(0.0, 0.0);
  const double2* Ap = A + p.a_off;
  for (int k0 = 0; k0 < p.k; k0 += TS_BK) {
    // A tile: 64 rows x 16 k, four elements per thread
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      int rr, kk;
      if (TRANS) {  // consecutive threads on consecutive k (contiguous in A^T's storage)
        kk = e % TS_BK;
        rr = e / TS_BK;
      } else {      // consecutive threads on consecutive rows
        rr = e % TS_BM;
        kk = e / TS_BM;
      }
      const int gr = m0 + rr, gk = k0 + kk;
      double2 v = make_double2(0.0, 0.0);
      if (gr < p.m && gk < p.k) v = TRANS ? Ap[gk + int64_t(gr) * p.lda] : Ap[gr + int64_t(gk) * p.lda];
      sa[kk][rr] = v;
    }
    {  // B tile: 16 rows x 16 columns, one element per thread
      const int kk = tid / EIG_NR, c = tid % EIG_NR;
      const int gk = k0 + kk;
      double2 v = make_double2(0.0, 0.0);
      if (gk < p.k) {
        const int64_t brow = GATHER ? int64_t(idx[p.b_off + gk]) : p.b_off + gk;
        v = B[brow * EIG_NR + c];
      }
      sb[kk][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TS_BK; ++kk) {
      const double2 a = sa[kk][row];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double2 b = sb[kk][4 * cg + j];
        acc[j].x += a.x * b.x - a.y * b.y;
        acc[j].y += a.x * b.y + a.y * b.x;
      }
    }
    __syncthreads();
  }
  const int gr = m0 + row;
  if (gr >= p.m) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = 4 * cg + j;
    double2 v = NEG ? make_double2(-acc[j].x, -acc[j].y) : acc[j];
    if (HAS_C0) {
      const double2 u = C0[(p.c0_off + gr) * EIG_NR + c];
      v.x += u.x;
      v.y += u.y;
    }
    C[(p.c_off + gr) * EIG_NR + c] = v;
  }
}

// V[v][c] = Re x[iperm[v]][c], V[v][EIG_NR + c] = Im x[iperm[v]][c]: the real
// basis of the Rayleigh-Ritz step, in the caller's order.
__global__ __launch_bounds__(256) void k_unperm_split(const double2* __restrict__ x, const int32_t* __restrict__ iperm,
                                                      int64_t n, double* __restrict__ v) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= n * EIG_NR) return;
  const int64_t r = t / EIG_NR;
  const int c = static_cast<int>(t % EIG_NR);
  const double2 u = x[int64_t(iperm[r]) * EIG_NR + c];
  v[r * 2 * EIG_NR + c] = u.x;
  v[r * 2 * EIG_NR + EIG_NR + c] = u.y;
}

// Partial Gram products of the projections (Eq. (B3)): part[b][i][j] =
// sum over rows v of chunk b of V[v][i] W[v][j], i, j < 2 EIG_NR; each of the
// 256 threads holds four (i, j) pairs; the host adds the chunks in order.
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ V, const double* __restrict__ W, int64_t n,
                                              int64_t chunk, double* __restrict__ part) {
  constexpr int NB = 2 * EIG_NR;
  const int64_t r0 = int64_t(blockIdx.x) * chunk;
  const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t r = r0; r < r1; ++r) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;
      s[q] += V[r * NB + e / NB] * W[r * NB + e % NB];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) part[int64_t(blockIdx.x) * NB * NB + threadIdx.x + 256 * q] = s[q];
}

// out[v][c] = sum_i V[v][i] Y[i][c] for c < EIG_NR (Ritz vectors from the
// basis and the coefficients of the small eigenproblem, 2 EIG_NR x EIG_NR).
__global__ __launch_bounds__(256) void k_combine(const double* __restrict__ V, const double* __restrict__ Y, int64_t n,
                                                 double* __restrict__ out) {
  constexpr int NB = 2 * EIG_NR;
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= n * EIG_NR) return;
  const int64_t r = t / EIG_NR;
  const int c = static_cast<int>(t % EIG_NR);
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NB; ++i) s += V[r * NB + i] * Y[i * EIG_NR + c];
  out[t] = s;
}

// part[b][c] = sum over rows of chunk b of (HC[v][c] - theta_c SC[v][c])^2
// (squared residual norms of the Ritz pairs).
__global__ __launch_bounds__(EIG_NR) void k_resid(const double* __restrict__ hc, const double* __restrict__ sc,
                                                  const double* __restrict__ theta, int64_t n, int64_t chunk,
                                                  double* __restrict__ part) {
  const int c = threadIdx.x;
  const int64_t r0 = int64_t(blockIdx.x) * chunk;
  const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;
  const double th = theta[c];
  double s = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const double d = hc[r * EIG_NR + c] - th * sc[r * EIG_NR + c];
    s += d * d;
  }
  part[int64_t(blockIdx.x) * EIG_NR + c] = s;
}

// ----------------------------------------------------------------- launchers

static inline unsigned nblocks(int64_t n, int per) { return static_cast<unsigned>((n + per - 1) / per); }

hipError_t launch_spmm_perm(const int64_t* rp, const int32_t* col, const double* a, const int32_t* perm, int64_t n,
                            const double* x, double2* y, hipStream_t st) {
  hipLaunchKernelGGL(k_spmm_perm, dim3(nblocks(n * EIG_NR, 256)), dim3(256), 0, st, rp, col, a, perm, n, x, y);
  return hipGetLastError();
}

hipError_t launch_spmm2(const int64_t* rp, const int32_t* col, const double* a, int64_t n, const double* x, double* w,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_spmm<2 * EIG_NR>, dim3(nblocks(n * 2 * EIG_NR, 256)), dim3(256), 0, st, rp, col, a, n, x, w);
  return hipGetLastError();
}

hipError_t launch_solve_gather(const SolveFront* fronts, const SolveChild* kids, const int32_t* inv,
                               const SolveTile* tiles, int64_t ntiles, const double2* y, double2* z, double2* w,
                               hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_solve_gather, dim3(static_cast<unsigned>(ntiles)), dim3(EIG_GROWS * EIG_NR), 0, st, fronts,
                     kids, inv, tiles, y, z, w);
  return hipGetLastError();
}

hipError_t launch_tsgemm(int mode, const TsProb* probs, const TsTile* tiles, int64_t ntiles, const double2* A,
                         const double2* B, const int32_t* idx, const double2* C0, double2* C, hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
  const dim3 g(static_cast<unsigned>(ntiles)), b(256);
  switch (mode) {
    case TS_FORWARD:   // w_f = w_f + L_f z_J
      hipLaunchKernelGGL((k_tsgemm<false, false, true, false>), g, b, 0, st, probs, tiles, A, B, idx, C0, C);
      break;
    case TS_DIAGONAL:  // z2_J = A_f^{-1} z_J
      hipLaunchKernelGGL((k_tsgemm<false, false, false, false>), g, b, 0, st, probs, tiles, A, B, idx, C0, C);
      break;
    case TS_BACKWARD:  // x_J = z2_J - L_f^T x_U
      hipLaunchKernelGGL((k_tsgemm<true, true, true, true>), g, b, 0, st, probs, tiles, A, B, idx, C0, C);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_unperm_split(const double2* x, const int32_t* iperm, int64_t n, double* v, hipStream_t st) {
  hipLaunchKernelGGL(k_unperm_split, dim3(nblocks(n * EIG_NR, 256)), dim3(256), 0, st, x, iperm, n, v);
  return hipGetLastError();
}

hipError_t launch_gram(const double* V, const double* W, int64_t n, int64_t chunk, int nblk, double* part,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_gram, dim3(static_cast<unsigned>(nblk)), dim3(256), 0, st, V, W, n, chunk, part);
  return hipGetLastError();
}

hipError_t launch_combine(const double* V, const double* Y, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_combine, dim3(nblocks(n * EIG_NR, 256)), dim3(256), 0, st, V, Y, n, out);
  return hipGetLastError();
}

hipError_t launch_resid(const double* hc, const double* sc, const double* theta, int64_t n, int64_t chunk, int nblk,
                        double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_resid, dim3(static_cast<unsigned>(nblk)), dim3(EIG_NR), 0, st, hc, sc, theta, n, chunk, part);
  return hipGetLastError();
}

}  // namespace ndrho
