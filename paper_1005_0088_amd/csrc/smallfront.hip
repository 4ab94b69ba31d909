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

// Shared memory of a workgroup: the staging of the products (a block of rows
// and a block of columns, SF_TK k each), which also holds the relative maps of
// the extend-add and the gather while no product runs.
constexpr int SF_STAGE = 160 * SF_TK;  // complex elements: (128 + 32) or (64 + 64) rows of SF_TK
constexpr int SF_MAXKIDS = 4;          // children whose maps are staged (more: read from global memory)
struct SfStage {
  double2 buf[SF_STAGE];
};

// out(r, c) = sum_k X(r, k) Y(k, c) for rows r0 .. r0 + R - 1 (r < m) and
// columns c0 .. c0 + C - 1 (c < nc), k < kk, with (R, C) = (128, 32) for
// narrow products (nc - c0 <= 32) and (64, 64) otherwise, so that pivot
// blocks of <= 32 rows do not compute 64 columns.  X and Y are read through
// the accessors (complex values), staged by SF_TK.  Thread tid owns row
// r0 + tid % R and the 16 columns c0 + 16 (tid / R) + j (acc[j]).
template <int R, class FX, class FY>
__device__ void block_product_t(double2 (&acc)[16], int r0, int m, int c0, int nc, int kk, FX X, FY Y,
                                SfStage& st) {
  constexpr int C = 4096 / R;  // 256 threads x 16 columns
  double2* sx = st.buf;            // [SF_TK][R]
  double2* sy = st.buf + SF_TK * R;  // [SF_TK][C]
  const int tid = threadIdx.x;
  const int row = tid % R, cb = tid / R;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < kk; k0 += SF_TK) {
#pragma unroll
    for (int q = 0; q < (SF_TK * R) / SF_THREADS; ++q) {
      const int e = tid + SF_THREADS * q;
      const int rr = e % R, k = e / R, gk = k0 + k;
      sx[k * R + rr] = (r0 + rr < m && gk < kk) ? X(r0 + rr, gk) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < (SF_TK * C) / SF_THREADS; ++q) {
      const int e = tid + SF_THREADS * q;
      const int cc = e % C, k = e / C, gk = k0 + k;
      sy[k * C + cc] = (c0 + cc < nc && gk < kk) ? Y(gk, c0 + cc) : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 1
    for (int k = 0; k < SF_TK; ++k) {
      const double2 x = sx[k * R + row];
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] = cmla(acc[j], x, sy[k * C + 16 * cb + j]);
    }
    __syncthreads();
  }
}

// Calls f(r, c, v) for every element of X Y (r < m, c < nc; rows from r_lo,
// columns from 0) with block shapes chosen by the product's width: blocks of
// 128 x 32 when nc <= 32, else 64 x 64.  With lower = true only blocks that
// hold an element with r >= c are formed (f still gets their upper ones).
template <class FX, class FY, class FO>
__device__ void product(int m, int nc, int kk, bool lower, FX X, FY Y, FO f, SfStage& st) {
  const int tid = threadIdx.x;
  double2 acc[16];
  if (nc <= 32) {
    for (int r0 = 0; r0 < m; r0 += 128) {
      block_product_t<128>(acc, r0, m, 0, nc, kk, X, Y, st);
      const int r = r0 + tid % 128, cb = tid / 128;
      if (r < m)
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (16 * cb + j < nc) f(r, 16 * cb + j, acc[j]);
    }
    return;
  }
  for (int c0 = 0; c0 < nc; c0 += 64)
    for (int r0 = lower ? c0 : 0; r0 < m; r0 += 64) {
      block_product_t<64>(acc, r0, m, c0, nc, kk, X, Y, st);
      const int r = r0 + tid % 64, cb = tid / 64;
      if (r < m)
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int c = c0 + 16 * cb + j;
          if (c < nc) f(r, c, acc[j]);
        }
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
  const int nj = F.nj, nu = F.nu, nm = nj + nu;
  const int64_t ld = nm;
  double2* pan = panel + p * ps + F.panel_off;
  double2* ucur = ((F.depth & 1) ? upd1 : upd0) + p * us;
  const double2* uch = ((F.depth & 1) ? upd0 : upd1) + p * us;
  // 1. the children's updates pulled onto the panel (columns J) and onto the
  //    front's own update block (lower triangle), children in order.  Their
  //    maps (front-local row -> child update row or -1) are staged in LDS
  //    first; each thread then issues the entry reads of four elements of a
  //    child together.
  const bool staged = F.child_count <= SF_MAXKIDS;
  int32_t* ims = reinterpret_cast<int32_t*>(st.buf);
  if (staged) {
    for (int e = tid; e < F.child_count * nm; e += SF_THREADS)
      ims[e] = inv[kids[F.child_begin + e / nm].inv_off + e % nm];
    __syncthreads();
  }
  auto pull = [&](int64_t total, int64_t rows, int roff, bool lower, double2* dst) {
    for (int64_t e0 = tid; e0 < total; e0 += 4 * SF_THREADS) {
      int rr[4], ss[4];
      bool in[4];
      double2 sum[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t e = e0 + int64_t(q) * SF_THREADS;
        rr[q] = static_cast<int>(e % rows) + roff;
        ss[q] = static_cast<int>(e / rows) + roff;
        in[q] = e < total && !(lower && rr[q] < ss[q]);
        sum[q] = make_double2(0.0, 0.0);
      }
      for (int c = 0; c < F.child_count; ++c) {
        const SmallChild k = kids[F.child_begin + c];
        const int32_t* im = staged ? ims + c * nm : inv + k.inv_off;
        int a[4], b[4];
        double2 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          a[q] = in[q] ? im[rr[q]] : -1;
          b[q] = in[q] ? im[ss[q]] : -1;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          v[q] = (a[q] >= 0 && b[q] >= 0) ? uch[k.upd_off + max(a[q], b[q]) + int64_t(min(a[q], b[q])) * k.nu]
                                          : make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (a[q] >= 0 && b[q] >= 0) {
            sum[q].x += v[q].x;
            sum[q].y += v[q].y;
          }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (in[q]) dst[e0 + int64_t(q) * SF_THREADS] = sum[q];
    }
  };
  pull(ld * nj, ld, 0, false, pan);
  pull(int64_t(nu) * nu, nu, nj, true, ucur + F.upd_off);
  __syncthreads();
  // 2. assembly of alpha S - h H at the front's table positions (four
  //    entries per thread at a time)
  for (int64_t k0 = F.asm_begin + tid; k0 < F.asm_end; k0 += 4 * SF_THREADS) {
    int64_t slot[4];
    double2 add[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t k = k0 + int64_t(q) * SF_THREADS;
      slot[q] = -1;
      if (k < F.asm_end) {
        slot[q] = asm_slot[k] - F.panel_off;
        const int32_t e = asm_entry[k];
        const double2 a = alpha[int64_t(asm_sid[k]) * astride + p];
        const double h = hcoef * hv[e], s = sv[e];
        add[q] = make_double2(a.x * s - h, a.y * s);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (slot[q] >= 0) {
        double2 v = pan[slot[q]];
        v.x += add[q].x;
        v.y += add[q].y;
        pan[slot[q]] = v;
      }
  }
  __syncthreads();
  // 3. pivot-block inverse (in place, symmetrized)
  pivot_inverse(pan, ld, nj, status, spd_check);
  if (nu == 0) return;
  // 4. L = B A^{-1} (nu x nj, ld nu)
  double2* L = lbuf + p * ls + F.l_off;
  product(nu, nj, nj, false, [&](int u, int k) { return pan[nj + u + int64_t(k) * ld]; },
          [&](int k, int j) { return pan[k + int64_t(j) * ld]; },
          [&](int u, int j, double2 v) { L[u + int64_t(j) * nu] = v; }, st);
  __syncthreads();
  // 5. Schur update of the lower triangle: Upd(r, s) -= sum_k L(r, k) B(s, k)
  double2* U = ucur + F.upd_off;
  product(nu, nu, nj, true, [&](int r, int k) { return L[r + int64_t(k) * nu]; },
          [&](int k, int s) { return pan[nj + s + int64_t(k) * ld]; },
          [&](int r, int s, double2 a) {
            if (r >= s) {
              double2 v = U[r + int64_t(s) * nu];
              v.x -= a.x;
              v.y -= a.y;
              U[r + int64_t(s) * nu] = v;
            }
          },
          st);
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
  if (nu == 0) return;
  double2* pan = panel + p * ps + F.panel_off;
  double2* guu = ((F.depth & 1) ? upd1 : upd0) + p * us + F.upd_off;
  if (F.parent_small) {
    // gather the lower triangle of G_UU from the parent's G (its panel and
    // its own G_UU) through the relative map, staged in LDS; four entries per
    // thread at a time
    int32_t* rl = reinterpret_cast<int32_t*>(st.buf);
    for (int a = tid; a < nu; a += SF_THREADS) rl[a] = rel[F.rel_off + a];
    __syncthreads();
    const double2* ppan = panel + p * ps + F.ppanel_off;
    const double2* pg = ((F.depth & 1) ? upd0 : upd1) + p * us + F.pguu_off;
    const int64_t pld = F.pnj + F.pnu, total = int64_t(nu) * nu;
    for (int64_t e0 = tid; e0 < total; e0 += 4 * SF_THREADS) {
      double2 v[4];
      bool in[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t e = e0 + int64_t(q) * SF_THREADS;
        const int a = static_cast<int>(e % nu), b = static_cast<int>(e / nu);
        in[q] = e < total && a >= b;
        const int r = in[q] ? rl[a] : 0, c = in[q] ? rl[b] : 0;
        v[q] = !in[q] ? make_double2(0.0, 0.0)
                      : c < F.pnj ? ppan[r + int64_t(c) * pld] : pg[(r - F.pnj) + int64_t(c - F.pnj) * F.pnu];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (in[q]) guu[e0 + int64_t(q) * SF_THREADS] = v[q];
    }
    __syncthreads();
  }
  const double2* L = lbuf + p * ls + F.l_off;
  // G_UJ = -G_UU L over the B rows of the panel (G_UU from its lower triangle)
  product(nu, nj, nu, false, [&](int u, int v) { return guu[max(u, v) + int64_t(min(u, v)) * nu]; },
          [&](int v, int j) { return L[v + int64_t(j) * nu]; },
          [&](int u, int j, double2 a) { pan[nj + u + int64_t(j) * ld] = make_double2(-a.x, -a.y); }, st);
  __syncthreads();
  // G_JJ = A^{-1} - L^T G_UJ: each lower element from the A^{-1} element its
  // own thread reads, then written with its mirror (no thread reads an upper
  // element; the product's staging reads only the B rows)
  product(nj, nj, nu, false, [&](int j, int u) { return L[u + int64_t(j) * nu]; },
          [&](int u, int j) { return pan[nj + u + int64_t(j) * ld]; },
          [&](int r, int c, double2 a) {
            if (r >= c) {
              const double2 x = pan[r + int64_t(c) * ld];
              const double2 g = make_double2(x.x - a.x, x.y - a.y);
              pan[r + int64_t(c) * ld] = g;
              if (r != c) pan[c + int64_t(r) * ld] = g;
            }
          },
          st);
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
