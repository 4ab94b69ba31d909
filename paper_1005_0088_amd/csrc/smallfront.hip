// Fused kernels of the small fronts (the deep levels of the dissection tree).
// One launch per depth and direction covers every small front of that depth
// for every pole of the pass, one workgroup per (front, pole).  Upward, a
// workgroup does the front's whole step: extend-add of its children's
// updates, assembly, pivot-block inverse, L = B A^{-1} and the Schur update
// (Eqs. (18)-(20)).  Downward it gathers G_UU from the parent and forms
// G_UJ = -G_UU L and G_JJ = A^{-1} - L^T G_UJ (Eqs. (21), (38)-(39)).  The
// depths are separate launches in tree order on one stream, so no workgroup
// ever waits for another.
//
// A small front has at most 64 pivot rows and, with its whole subtree, fits
// the plan's bound on pivot plus update rows; each has an update block of its
// own.  All arithmetic is FP64.  A host build of this file through a stand-in
// HIP header reproduces the selected inverse (tests/test_small_schedule_emu.py).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace ndrho {

namespace {

constexpr int SF_THREADS = 256;
constexpr int SF_TK = 16;  // k staged per step of the products

__device__ __forceinline__ double2 cmla(double2 acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
  return acc;
}

// In-place Gauss-Jordan inverse of the n x n (n <= 64) symmetric pivot block
// at a (leading dimension ld), without pivoting, by the whole workgroup: as
// the pivot-inverse kernel (register rows, the pivot row broadcast through
// LDS, a_rk = -a_kr for r < k and a_kr otherwise), pivots checked the same way.
__device__ void pivot_inverse(double2* a, int64_t ld, int n, int* status, int spd_check) {
  constexpr int NMAX = 64, CG = SF_THREADS / NMAX, COLS = NMAX / CG;
  __shared__ double2 rowk[2][NMAX];
  __shared__ double dmag[NMAX];
  __shared__ double sdiag_s;
  const int tid = threadIdx.x;
  const int r = tid % NMAX, cg = tid / NMAX;
  const bool live = r < n;
  double2 v[COLS];
#pragma unroll
  for (int i = 0; i < COLS; ++i) {
    const int c = cg + CG * i;
    v[i] = make_double2(0.0, 0.0);
    if (live && c < n) v[i] = a[r + int64_t(c) * ld];
  }
  if (tid < n) {
    const double2 x = a[tid + int64_t(tid) * ld];
    dmag[tid] = fabs(x.x) + fabs(x.y);
  }
  __syncthreads();
  if (tid == 0) {
    double sd = 0.0;
    for (int i = 0; i < n; ++i) sd = fmax(sd, dmag[i]);
    sdiag_s = sd;
  }
  __syncthreads();
  const double sdiag = sdiag_s;
  int bad_sing = 0, bad_spd = 0;
  for (int k = 0; k < n; ++k) {
    const int b = k & 1;
    if (r == k) {
#pragma unroll
      for (int i = 0; i < COLS; ++i) {
        const int c = cg + CG * i;
        if (c < n) rowk[b][c] = v[i];
      }
    }
    __syncthreads();
    const double2 p = rowk[b][k];
    if (tid == 0) {
      const double mag = fabs(p.x) + fabs(p.y);
      if (!(mag > 1e-14 * sdiag) || !isfinite(p.x) || !isfinite(p.y)) bad_sing = 1;
      if (spd_check && !(p.x > 0.0 && p.y == 0.0)) bad_spd = 1;
    }
    const double s = fmax(fabs(p.x), fabs(p.y));
    const double xr = p.x / s, xi = p.y / s;
    const double dd = (xr * xr + xi * xi) * s;
    const double2 pinv = make_double2(xr / dd, -xi / dd);
    const double2 akr = rowk[b][r];
    const double sg = r < k ? -1.0 : 1.0;
    const bool prow = r == k;
    const double2 sa = make_double2(sg * akr.x, sg * akr.y);
    const double2 fr = make_double2(sa.x * pinv.x - sa.y * pinv.y, sa.x * pinv.y + sa.y * pinv.x);
    const double2 f = prow ? make_double2(-pinv.x, -pinv.y) : fr;
    const double keep = prow ? 0.0 : 1.0;
    const double2 colk = prow ? pinv : make_double2(-fr.x, -fr.y);
#pragma unroll
    for (int i = 0; i < COLS; ++i) {
      const int c = cg + CG * i;
      const double2 rk = rowk[b][c];
      const double ux = keep * v[i].x - (f.x * rk.x - f.y * rk.y);
      const double uy = keep * v[i].y - (f.x * rk.y + f.y * rk.x);
      const bool ck = c == k;
      v[i].x = ck ? colk.x : ux;
      v[i].y = ck ? colk.y : uy;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < COLS; ++i) {
    const int c = cg + CG * i;
    if (live && c < n && r >= c) {
      a[r + int64_t(c) * ld] = v[i];
      if (r != c) a[c + int64_t(r) * ld] = v[i];
    }
  }
  if (tid == 0) {
    if (bad_sing) atomicAdd(&status[0], 1);
    if (bad_spd) atomicAdd(&status[1], 1);
  }
  __syncthreads();
}

// Shared staging of the products: two 64 x SF_TK complex tiles.
struct SfStage {
  double2 x[SF_TK][64];
  double2 y[SF_TK][64];
};

// out[r][c] (r < m rows, c < nc <= 64 columns) = sum_k X(r, k) Y(k, c) for a
// 64-row block starting at row r0, k < kk; X and Y are read through the
// accessors (complex values), staged by SF_TK.  Thread (tid % 64) owns row
// r0 + tid % 64 and the 16 columns 16 (tid / 64) + j; acc holds them.
template <class FX, class FY>
__device__ void block_product(double2 (&acc)[16], int r0, int m, int nc, int kk, FX X, FY Y, SfStage& st) {
  const int tid = threadIdx.x;
  const int row = tid % 64, cb = tid / 64;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < kk; k0 += SF_TK) {
#pragma unroll
    for (int q = 0; q < (SF_TK * 64) / SF_THREADS; ++q) {
      const int e = tid + SF_THREADS * q;
      const int rr = e % 64, k = e / 64;
      const int gk = k0 + k;
      st.x[k][rr] = (r0 + rr < m && gk < kk) ? X(r0 + rr, gk) : make_double2(0.0, 0.0);
      st.y[k][rr] = (rr < nc && gk < kk) ? Y(gk, rr) : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 1
    for (int k = 0; k < SF_TK; ++k) {
      const double2 x = st.x[k][row];
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] = cmla(acc[j], x, st.y[k][16 * cb + j]);
    }
    __syncthreads();
  }
}

}  // namespace

// Upward step of one small front for one pole (workgroup b of the launch:
// front b / npoles of the depth's list, pole b % npoles).  The fronts of the
// next deeper depth (its children) finished in the launch before.  The update
// blocks of the front's depth and of its children's depth are in upd0 / upd1
// by depth parity (pole p at + p * us).
__global__ __launch_bounds__(SF_THREADS, 2) void k_small_up(
    const SmallFront* __restrict__ fronts, const SmallChild* __restrict__ kids, const int32_t* __restrict__ inv,
    int npoles, double2* panel, int64_t ps, double2* lbuf, int64_t ls, double2* upd0, double2* upd1, int64_t us,
    const int64_t* __restrict__ asm_slot, const int32_t* __restrict__ asm_entry, const int32_t* __restrict__ asm_sid,
    const double* __restrict__ hv, const double* __restrict__ sv, const double2* __restrict__ alpha, int64_t astride,
    double hcoef, int spd_check, int* status) {
  __shared__ SfStage st;
  const int tid = threadIdx.x;
  const int64_t fi = blockIdx.x / npoles;
  const int p = static_cast<int>(blockIdx.x % npoles);
  const SmallFront F = fronts[fi];
  const int nj = F.nj, nu = F.nu;
  const int64_t ld = nj + nu;
  double2* pan = panel + p * ps + F.panel_off;
  double2* ucur = ((F.depth & 1) ? upd1 : upd0) + p * us;
  const double2* uch = ((F.depth & 1) ? upd0 : upd1) + p * us;
  // 1. the children's updates pulled onto the panel (columns J) and onto
  //    the front's own update block (lower triangle), children in order
  const int64_t np_ = ld * nj;
  for (int64_t e = tid; e < np_; e += SF_THREADS) {
    const int r = static_cast<int>(e % ld), s = static_cast<int>(e / ld);
    double2 sum = make_double2(0.0, 0.0);
    for (int c = 0; c < F.child_count; ++c) {
      const SmallChild k = kids[F.child_begin + c];
      const int32_t* im = inv + k.inv_off;
      const int a = im[r], b = im[s];
      if (a >= 0 && b >= 0) {
        const double2 v = uch[k.upd_off + max(a, b) + int64_t(min(a, b)) * k.nu];
        sum.x += v.x;
        sum.y += v.y;
      }
    }
    pan[e] = sum;
  }
  const int64_t nuu = int64_t(nu) * nu;
  for (int64_t e = tid; e < nuu; e += SF_THREADS) {
    const int r = static_cast<int>(e % nu), s = static_cast<int>(e / nu);
    if (r < s) continue;
    double2 sum = make_double2(0.0, 0.0);
    for (int c = 0; c < F.child_count; ++c) {
      const SmallChild k = kids[F.child_begin + c];
      const int32_t* im = inv + k.inv_off;
      const int a = im[nj + r], b = im[nj + s];
      if (a >= 0 && b >= 0) {
        const double2 v = uch[k.upd_off + max(a, b) + int64_t(min(a, b)) * k.nu];
        sum.x += v.x;
        sum.y += v.y;
      }
    }
    ucur[F.upd_off + e] = sum;
  }
  __syncthreads();
  // 2. assembly of alpha S - h H at the front's table positions
  for (int64_t k = F.asm_begin + tid; k < F.asm_end; k += SF_THREADS) {
    const int64_t slot = asm_slot[k] - F.panel_off;
    const int32_t e = asm_entry[k];
    const double2 a = alpha[int64_t(asm_sid[k]) * astride + p];
    const double h = hcoef * hv[e], s = sv[e];
    double2 v = pan[slot];
    v.x += a.x * s - h;
    v.y += a.y * s;
    pan[slot] = v;
  }
  __syncthreads();
  // 3. pivot-block inverse (in place, symmetrized)
  pivot_inverse(pan, ld, nj, status, spd_check);
  if (nu > 0) {
    // 4. L = B A^{-1} (nu x nj, ld nu)
    double2* L = lbuf + p * ls + F.l_off;
    const int row = tid % 64, cb = tid / 64;
    for (int u0 = 0; u0 < nu; u0 += 64) {
      double2 acc[16];
      block_product(acc, u0, nu, nj, nj, [&](int u, int k) { return pan[nj + u + int64_t(k) * ld]; },
                    [&](int k, int j) { return pan[k + int64_t(j) * ld]; }, st);
      const int u = u0 + row;
      if (u < nu)
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (16 * cb + j < nj) L[u + int64_t(16 * cb + j) * nu] = acc[j];
    }
    __syncthreads();
    // 5. Schur update of the lower triangle: Upd(r, s) -= sum_k L(r, k) B(s, k)
    for (int s0 = 0; s0 < nu; s0 += 64) {
      for (int r0 = s0; r0 < nu; r0 += 64) {
        double2 acc[16];
        block_product(acc, r0, nu, min(64, nu - s0), nj, [&](int r, int k) { return L[r + int64_t(k) * nu]; },
                      [&](int k, int s) { return pan[nj + s0 + s + int64_t(k) * ld]; }, st);
        const int r = r0 + row;
        if (r < nu)
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            const int s = s0 + 16 * cb + j;
            if (s < nu && r >= s) {
              double2 v = ucur[F.upd_off + r + int64_t(s) * nu];
              v.x -= acc[j].x;
              v.y -= acc[j].y;
              ucur[F.upd_off + r + int64_t(s) * nu] = v;
            }
          }
      }
    }
  }
}

// Downward step of one small front for one pole.  A small parent finished in
// the launch before; a large parent's level gathered this front's G_UU.
__global__ __launch_bounds__(SF_THREADS, 2) void k_small_down(
    const SmallFront* __restrict__ fronts, const int32_t* __restrict__ rel, int npoles, double2* panel, int64_t ps,
    const double2* __restrict__ lbuf, int64_t ls, double2* upd0, double2* upd1, int64_t us) {
  __shared__ SfStage st;
  const int tid = threadIdx.x;
  const int64_t fi = blockIdx.x / npoles;
  const int p = static_cast<int>(blockIdx.x % npoles);
  const SmallFront F = fronts[fi];
  const int nj = F.nj, nu = F.nu;
  const int64_t ld = nj + nu;
  double2* pan = panel + p * ps + F.panel_off;
  double2* guu = ((F.depth & 1) ? upd1 : upd0) + p * us + F.upd_off;
  if (nu > 0) {
    if (F.parent_small) {
      // gather the lower triangle of G_UU from the parent's G (its panel
      // and its own G_UU), through the relative map
      const int32_t* rl = rel + F.rel_off;
      const double2* ppan = panel + p * ps + F.ppanel_off;
      const double2* pg = ((F.depth & 1) ? upd0 : upd1) + p * us + F.pguu_off;
      const int64_t pld = F.pnj + F.pnu;
      for (int64_t e = tid; e < int64_t(nu) * nu; e += SF_THREADS) {
        const int a = static_cast<int>(e % nu), b = static_cast<int>(e / nu);
        if (a < b) continue;
        const int r = rl[a], s = rl[b];
        guu[e] = s < F.pnj ? ppan[r + int64_t(s) * pld] : pg[(r - F.pnj) + int64_t(s - F.pnj) * F.pnu];
      }
      __syncthreads();
    }
    const double2* L = lbuf + p * ls + F.l_off;
    const int row = tid % 64, cb = tid / 64;
    // G_UJ = -G_UU L over the B rows of the panel (G_UU from its lower triangle)
    for (int u0 = 0; u0 < nu; u0 += 64) {
      double2 acc[16];
      block_product(acc, u0, nu, nj, nu,
                    [&](int u, int v) { return guu[max(u, v) + int64_t(min(u, v)) * nu]; },
                    [&](int v, int j) { return L[v + int64_t(j) * nu]; }, st);
      const int u = u0 + row;
      if (u < nu)
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (16 * cb + j < nj) pan[nj + u + int64_t(16 * cb + j) * ld] = make_double2(-acc[j].x, -acc[j].y);
    }
    __syncthreads();
    // G_JJ = A^{-1} - L^T G_UJ: each lower element from the A^{-1} element
    // its own thread reads, then written with its mirror (no thread reads
    // an upper element)
    double2 acc[16];
    block_product(acc, 0, nj, nj, nu, [&](int j, int u) { return L[u + int64_t(j) * nu]; },
                  [&](int u, int j) { return pan[nj + u + int64_t(j) * ld]; }, st);
    if (row < nj)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int c = 16 * cb + j;
        if (c < nj && row >= c) {
          const double2 a = pan[row + int64_t(c) * ld];
          const double2 g = make_double2(a.x - acc[j].x, a.y - acc[j].y);
          pan[row + int64_t(c) * ld] = g;
          if (row != c) pan[c + int64_t(row) * ld] = g;
        }
      }
  }
}

hipError_t launch_small(const SmallLaunch& s, hipStream_t st) {
  if (s.nfronts == 0) return hipSuccess;
  const int64_t ntasks = s.nfronts * s.npoles;
  if (ntasks > 0x7FFFFFFF) return hipErrorInvalidValue;
  const unsigned grid = static_cast<unsigned>(ntasks);
  if (s.up)
    hipLaunchKernelGGL(k_small_up, dim3(grid), dim3(SF_THREADS), 0, st, s.fronts, s.kids, s.inv, s.npoles, s.panel,
                       s.ps, s.lbuf, s.ls, s.upd0, s.upd1, s.us, s.asm_slot, s.asm_entry, s.asm_sid, s.hv, s.sv,
                       s.alpha, s.astride, s.hcoef, s.spd_check, s.status);
  else
    hipLaunchKernelGGL(k_small_down, dim3(grid), dim3(SF_THREADS), 0, st, s.fronts, s.rel, s.npoles, s.panel, s.ps,
                       s.lbuf, s.ls, s.upd0, s.upd1, s.us);
  return hipGetLastError();
}

}  // namespace ndrho
