// Device kernels of the front-by-front block LDL^T factorization and selected
// inversion (Sec. II C 2, Eqs. (18)-(21), (38)-(39)) and of the pole sum of
// Eq. (8), for gfx950.  Complex numbers are interleaved (re, im) doubles;
// every per-pole buffer is laid out as [pole][elements] with a pole stride.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace ndrho {

typedef double d4 __attribute__((ext_vector_type(4)));

// Row of the 16x16 accumulator held in register r by `lane` (columns are
// lane % 16), as measured on gfx950: f64 16x16x4 interleaves the rows
// (4r + lane/16), f32 16x16x4 keeps them in blocks of four (4 (lane/16) + r).
#define F64_DROW(r, lane) (4 * (r) + ((lane) >> 4))
#define F32_DROW(r, lane) (4 * ((lane) >> 4) + (r))

// ----------------------------------------------------------------- helpers

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// 1/p = conj(p) / |p|^2 with one division: p is first scaled exactly by the
// power of two that brings its larger part into [0.5, 1), so that |p|^2
// neither overflows nor underflows, and the result is scaled back.
__device__ __forceinline__ double2 cinv(double2 p) {
  int e;
  frexp(fmax(fabs(p.x), fabs(p.y)), &e);
  const double xr = ldexp(p.x, -e), xi = ldexp(p.y, -e);
  const double t = 1.0 / (xr * xr + xi * xi);
  return make_double2(ldexp(xr * t, -e), ldexp(-xi * t, -e));
}

// Element i of a GEMM's A operand: FP64 complex, or FP32 complex widened
// exactly (G_A32; the low-precision products round it to FP32 in any case).
template <bool A32>
__device__ __forceinline__ double2 a_elem(const double2* Ap, int64_t i) {
  if (A32) {
    const float2 x = reinterpret_cast<const float2*>(Ap)[i];
    return make_double2(static_cast<double>(x.x), static_cast<double>(x.y));
  }
  return Ap[i];
}

// Blocks of a launch are dealt to the 8 XCDs round-robin by linear id; this
// remap gives every XCD one contiguous range of logical work items, so the
// tiles of one pole (which share operand panels) meet in one L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t total) {
  const int64_t x = b % 8, local = b / 8, q = total / 8, r = total % 8;
  return x * q + (x < r ? x : r) + local;
}

// Relative maps of a G_EXTC0 tile staged in LDS: for each child c of the
// front (at most XM_MAX), the child-local update index (or -1) of the tile's
// rows m0 .. m0 + tile - 1 at [c][0 .. tile) and of its columns n0 ..
// n0 + tile - 1 at [c][tile .. 2 tile).  p == nullptr: not staged (a front
// with more children, or a kernel without LDS); the epilogue then reads the
// maps from global memory.
constexpr int XM_MAX = 4;
struct XMap {
  const int32_t* p;
  int m0, n0, tile;
};

// Copies the maps of the tile's children into LDS (`mem`, at least
// 2 * XM_MAX * tile int32) once the main loop has finished with it: every
// kernel's K loop ends on a barrier after its last read of the staging
// memory, so the copy may start at once; a barrier follows it.  Called by the
// whole workgroup (the child count is uniform).
template <int NT>
__device__ __forceinline__ XMap stage_ext_maps(void* mem, int tile, const GemmProb& pr, const ExtAddDesc& xd,
                                               const ExtAddChild* __restrict__ xk, const int32_t* __restrict__ xi,
                                               int m0, int n0) {
  if (xd.child_count > XM_MAX) return XMap{nullptr, m0, n0, tile};
  int32_t* xm = static_cast<int32_t*>(mem);
  const int per = 2 * tile;
  for (int e = threadIdx.x; e < xd.child_count * per; e += NT) {
    const int c = e / per, w = e % per;
    const bool col = w >= tile;
    const int pos = (col ? n0 : m0) + (col ? w - tile : w);
    const ExtAddChild k = xk[xd.child_begin + c];
    xm[e] = pos < (col ? pr.n : pr.m) ? xi[k.inv_off + xd.nj + pos] : -1;
  }
  __syncthreads();
  return XMap{xm, m0, n0, tile};
}

// Epilogue of a chunk of NE result elements held by one thread,
// C = [C0 +] (+/-) product: negate, add C0 (read from memory with G_BETA,
// formed from the children with G_EXTC0), store, and with a mirrored
// symmetric output store the transpose too.  Elements outside the problem, or
// above the diagonal of a symmetric output, are skipped.  With G_EXTC0 the C0
// of an element of a front's U x U update is the sum, in child order, of the
// children's lower-stored update entries that map onto it (the same sum the
// extend-add forms for the panel).  With the maps staged in LDS (xm.p), the
// entry reads of two children are issued together, so that a thread waits
// once per pair of children; otherwise the map reads of the whole chunk are
// issued before any of its value reads (two waits per child).
template <int FLAGS, int NE>
__device__ __forceinline__ void store_chunk(double2 (&v)[NE], const int (&m)[NE], const int (&n)[NE],
                                            const GemmProb& pr, const double2* C0p, double2* Cp,
                                            const ExtAddDesc& xd, const ExtAddChild* __restrict__ xk,
                                            const int32_t* __restrict__ xi, const XMap& xm) {
  constexpr bool BETA = (FLAGS & G_BETA) != 0, NEG = (FLAGS & G_NEG) != 0, EXTC0 = (FLAGS & G_EXTC0) != 0;
  constexpr bool SYM = (FLAGS & G_SYM) != 0, MIRROR = SYM && !(FLAGS & G_NOMIRROR);
  bool live[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) live[q] = m[q] < pr.m && n[q] < pr.n && !(SYM && m[q] < n[q]);
  double2 c0[NE];
  if (EXTC0) {
#pragma unroll
    for (int q = 0; q < NE; ++q) c0[q] = make_double2(0.0, 0.0);
    if (xm.p) {
      for (int c = 0; c < xd.child_count; c += 2) {
        const bool two = c + 1 < xd.child_count;
        const ExtAddChild k0 = xk[xd.child_begin + c];
        const ExtAddChild k1 = xk[xd.child_begin + (two ? c + 1 : c)];
        const int32_t* r0 = xm.p + c * 2 * xm.tile;
        const int32_t* r1 = r0 + 2 * xm.tile;
        double2 x0[NE], x1[NE];
        bool ok0[NE], ok1[NE];
#pragma unroll
        for (int q = 0; q < NE; ++q) {
          const int a0 = live[q] ? r0[m[q] - xm.m0] : -1, b0 = live[q] ? r0[xm.tile + n[q] - xm.n0] : -1;
          const int a1 = live[q] && two ? r1[m[q] - xm.m0] : -1;
          const int b1 = live[q] && two ? r1[xm.tile + n[q] - xm.n0] : -1;
          ok0[q] = a0 >= 0 && b0 >= 0;
          ok1[q] = a1 >= 0 && b1 >= 0;
          // the children store the lower triangle of their update
          x0[q] = ok0[q] ? C0p[k0.upd_off + max(a0, b0) + int64_t(min(a0, b0)) * k0.nu] : make_double2(0.0, 0.0);
          x1[q] = ok1[q] ? C0p[k1.upd_off + max(a1, b1) + int64_t(min(a1, b1)) * k1.nu] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int q = 0; q < NE; ++q) {
          if (ok0[q]) {
            c0[q].x += x0[q].x;
            c0[q].y += x0[q].y;
          }
          if (ok1[q]) {
            c0[q].x += x1[q].x;
            c0[q].y += x1[q].y;
          }
        }
      }
    } else {
      for (int c = 0; c < xd.child_count; ++c) {
        const ExtAddChild k = xk[xd.child_begin + c];
        const int32_t* im = xi + k.inv_off + xd.nj;
        int32_t a[NE], b[NE];
#pragma unroll
        for (int q = 0; q < NE; ++q) {
          a[q] = live[q] ? im[m[q]] : -1;
          b[q] = live[q] ? im[n[q]] : -1;
        }
#pragma unroll
        for (int q = 0; q < NE; ++q)
          if (a[q] >= 0 && b[q] >= 0) {  // the children store the lower triangle of their update
            const double2 x = C0p[k.upd_off + max(a[q], b[q]) + int64_t(min(a[q], b[q])) * k.nu];
            c0[q].x += x.x;
            c0[q].y += x.y;
          }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    if (!live[q]) continue;
    double2 x = v[q];
    if (NEG) x = make_double2(-x.x, -x.y);
    if (BETA || EXTC0) {
      const double2 y = BETA ? C0p[m[q] + int64_t(n[q]) * pr.ldc0] : c0[q];
      x.x += y.x;
      x.y += y.y;
    }
    Cp[m[q] + int64_t(n[q]) * pr.ldc] = x;
    if (MIRROR && m[q] != n[q]) Cp[n[q] + int64_t(m[q]) * pr.ldc] = x;
  }
}

// ----------------------------------------------------------------- extend-add
//
// Pull form of the child-to-parent accumulation of Schur complements
// (Eq. (32); the (B[C])^T bookkeeping of Eq. (28)): every element of the
// parent's panel (columns in J) is written once as the sum, in child order,
// of the children's update entries that map onto it (update blocks are
// symmetric and stored as lower triangles; the relative maps are increasing,
// so lower maps to lower).  Writing (not adding) also clears the panel
// before assembly, so no separate fill is needed and no two threads touch
// one target.  The parent's own U x U block takes the same sum in the
// epilogue of its Schur-update GEMM (G_EXTC0).  Elements of the pivot block
// above its diagonal 64 x 64 blocks are skipped: the recursive pivot inverse
// reads only the lower part and the diagonal blocks, and writes the rest
// (as the mirror of its lower part) before anything reads it.
__global__ __launch_bounds__(256) void k_extadd(const ExtAddDesc* __restrict__ descs,
                                                const ExtAddChild* __restrict__ kids,
                                                const int32_t* __restrict__ inv, const ElemTile* __restrict__ tiles,
                                                int64_t ntiles, double2* __restrict__ panel, int64_t ps,
                                                const double2* __restrict__ cupd, int64_t cs) {
  const int64_t pole = blockIdx.y;
  const ElemTile t = tiles[blockIdx.x];
  const ExtAddDesc d = descs[t.desc];
  // per-front element counts stay far below 2^31: 32-bit index arithmetic
  const uint32_t ld = d.nj + d.nu;
  const uint32_t tp = ld * d.nj;
  double2* pan = panel + pole * ps + d.panel_off;
  const double2* cu = cupd + pole * cs;
  // four elements per thread; the map reads of all four are issued before
  // any value read, child by child (the sums keep the child order)
  uint32_t r[4], s[4];
  bool live[4];
  double2 sum[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t e = uint32_t(t.e0) + threadIdx.x + 256 * i;
    s[i] = e / ld;
    r[i] = e - s[i] * ld;
    // skipped: past the panel, or above the diagonal 64 x 64 blocks of the pivot block
    live[i] = e < tp && r[i] >= (s[i] & ~63u);
    sum[i] = make_double2(0.0, 0.0);
  }
  for (int c = 0; c < d.child_count; ++c) {
    const ExtAddChild k = kids[d.child_begin + c];
    const int32_t* im = inv + k.inv_off;
    int32_t a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = live[i] ? im[r[i]] : -1;
      b[i] = live[i] ? im[s[i]] : -1;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (a[i] >= 0 && b[i] >= 0) {  // children store the lower triangle of their update
        const double2 v = cu[k.upd_off + max(a[i], b[i]) + int64_t(min(a[i], b[i])) * k.nu];
        sum[i].x += v.x;
        sum[i].y += v.y;
      }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (live[i]) pan[r[i] + int64_t(s[i]) * ld] = sum[i];
}

// ----------------------------------------------------------------- assembly
//
// X = alpha_p S - h H for every pole of the batch, added into the panels at
// the table positions (each position receives at most one entry).  With
// several structures in one plan, entry k belongs to structure sid[k] and
// takes its shifts from alpha[sid[k] * astride + p].
__global__ __launch_bounds__(256) void k_assemble(const int64_t* __restrict__ slot, const int32_t* __restrict__ entry,
                                                  const int32_t* __restrict__ sid, int64_t count,
                                                  const double* __restrict__ hv, const double* __restrict__ sv,
                                                  const double2* __restrict__ alpha, int64_t astride, int npoles,
                                                  double hcoef, double2* __restrict__ panel, int64_t ps) {
  const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (k >= count) return;
  const int64_t sl = slot[k];
  const int32_t e = entry[k];
  const double h = hcoef * hv[e], s = sv[e];
  const double2* al = alpha + int64_t(sid[k]) * astride;
  for (int p = 0; p < npoles; ++p) {
    const double2 a = al[p];
    double2* x = panel + int64_t(p) * ps + sl;
    double2 v = *x;
    v.x += a.x * s - h;
    v.y += a.y * s;
    *x = v;
  }
}

// ----------------------------------------------------------------- pivot inverse
//
// In-place inverse of an n x n (n <= NMAX) symmetric pivot block by
// Gauss-Jordan elimination without pivoting, one workgroup per (block, pole).
// Size classes: NMAX = 64 on 512 threads, 32 on 128 and 16 on one wave.
// Thread t owns row r = t % NMAX and the columns c = t / NMAX + CG i
// (CG = THREADS / NMAX column groups, i < NMAX / CG) in registers.  Step k publishes row k through LDS; column k is not needed
// separately: for a symmetric start, after the pivots 0..k-1 have been
// eliminated an entry between an eliminated and a remaining index equals
// minus its transpose and all others equal their transpose, so
// a_rk = -a_kr for r < k and a_rk = a_kr otherwise.  The pivots met are the
// D of the block's LDL^T (Eq. (18)): |d| <= 1e-14 max|a_ii| or non-finite
// counts as singular; with spd_check a pivot with d <= 0 or Im d != 0 counts
// as "not positive definite" (the real factorization of S).  The result is
// written symmetrized from its lower triangle.
template <int NMAX, int THREADS>
__global__ __launch_bounds__(THREADS) void k_smallinv(const InvDesc* __restrict__ descs, double2* __restrict__ panel,
                                                      int64_t ps, int* __restrict__ status, int spd_check) {
  constexpr int CG = THREADS / NMAX, COLS = NMAX / CG;
  static_assert(CG * NMAX == THREADS && CG * COLS == NMAX, "size class");
  __shared__ double2 rowk[2][NMAX];
  __shared__ double dmag[NMAX];
  const InvDesc d = descs[blockIdx.x];
  const int n = d.n;
  const int64_t ld = d.ld;
  double2* a = panel + int64_t(blockIdx.y) * ps + d.off;
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
  double sdiag = 0.0;
  if (tid == 0)
    for (int i = 0; i < n; ++i) sdiag = fmax(sdiag, dmag[i]);
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
    const double2 pinv = cinv(p);
    const double2 akr = rowk[b][r];
    const double sg = r < k ? -1.0 : 1.0;  // a_rk = sg * a_kr
    const bool prow = r == k;
    // every element takes a_rc <- keep a_rc - f_r a_kc: off the pivot row
    // keep = 1 and f_r = a_rk / a_kk (the rank-1 update); on it keep = 0 and
    // f_k = -1/a_kk, which is the scaling of the pivot row by 1/a_kk.  The
    // column k becomes -f_r (1/a_kk on the pivot row).  Rows r >= n and
    // columns c >= n compute garbage that is never stored or published.
    const double2 fr = cmul(make_double2(sg * akr.x, sg * akr.y), pinv);
    const double2 f = prow ? make_double2(-pinv.x, -pinv.y) : fr;
    const double keep = prow ? 0.0 : 1.0;
    const double2 colk = prow ? pinv : make_double2(-fr.x, -fr.y);
#pragma unroll
    for (int i = 0; i < COLS; ++i) {
      const int c = cg + CG * i;
      const double2 rk = rowk[b][c];
      // (selects on scalars: a select of double2 values goes through memory)
      const double ux = keep * v[i].x - (f.x * rk.x - f.y * rk.y);
      const double uy = keep * v[i].y - (f.x * rk.y + f.y * rk.x);
      const bool ck = c == k;
      v[i].x = ck ? colk.x : ux;
      v[i].y = ck ? colk.y : uy;
    }
  }
  // symmetrized write-back from the lower triangle
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
}

// ----------------------------------------------------------------- complex GEMM
//
// C = [C0 +] (+/-) op(A) op(B), grouped over problems and batched over poles,
// complex FP64 on the matrix cores (v_mfma_f64_16x16x4f64).  Each complex
// product takes three real ones (P1 = Ar Br, P2 = Ai Bi, P3 = (Ar+Ai)(Br+Bi);
// Re = P1 - P2, Im = P3 - P1 - P2), issued so that consecutive MFMAs never
// share an accumulator.  Transposes are plain transposes (the matrices are
// complex symmetric, never Hermitian).  One 64x64 output tile per workgroup
// of eight waves (2 x 4 waves of 32 x 16, a third of the accumulators per
// wave, so that two workgroups per compute unit give four waves per SIMD and
// hide one another's LDS and barrier waits), K staged through LDS in steps of
// 16 with double buffering.  The MFMA operands are swapped (B-tile as the A
// operand) so that each lane owns one row of C (the accumulator of the f64
// 16x16x4 instruction holds D[4r + lane/16][lane%16] in register r), and a
// wave's stores run down the columns of the column-major C.  With G_SYM only tiles
// on or below the diagonal are computed and each lower element is also
// written to its mirror, so symmetric results stay exactly symmetric.
constexpr int BM = 64, BN = 64, BK = 16;

template <int FLAGS>
__global__ __launch_bounds__(512, 4) void k_zgemm(const GemmProb* __restrict__ probs,
                                                  const TileRef* __restrict__ tiles, int64_t ntiles, int64_t npoles,
                                                  const double2* __restrict__ A, int64_t sA,
                                                  const double2* __restrict__ B, int64_t sB, const double2* C0,
                                                  int64_t sC0, double2* C, int64_t sC,
    const ExtAddDesc* __restrict__ xe, const ExtAddChild* __restrict__ xk, const int32_t* __restrict__ xi) {
  constexpr bool TA = (FLAGS & G_TA) != 0, TB = (FLAGS & G_TB) != 0;
  constexpr bool BETA = (FLAGS & G_BETA) != 0, EXTC0 = (FLAGS & G_EXTC0) != 0;
  constexpr bool SYMA = (FLAGS & G_SYMA) != 0, A32 = (FLAGS & G_A32) != 0;
  static_assert(!(SYMA && TA), "a lower-stored symmetric A is read untransposed");
  static_assert(!A32, "the FP64 kernels read FP64 operands");
  __shared__ double2 As[2][BK][BM + 1];
  __shared__ double2 Bs[2][BK][BN + 1];

  const int64_t total = ntiles * npoles;
  const int64_t logical = xcd_remap(blockIdx.x, total);
  const int64_t pole = logical / ntiles;
  const TileRef tr = tiles[logical % ntiles];
  const GemmProb pr = probs[tr.prob];
  const double2* Ap = A + pole * sA + pr.a_off;
  const double2* Bp = B + pole * sB + pr.b_off;
  const int M = pr.m, N = pr.n, K = pr.k;
  const int m0 = tr.tm * BM, n0 = tr.tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;   // wave piece: rows 32 wm.., columns 16 wn..

  d4 p1[2], p2[2], p3[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    p1[i] = d4{0.0, 0.0, 0.0, 0.0};
    p2[i] = d4{0.0, 0.0, 0.0, 0.0};
    p3[i] = d4{0.0, 0.0, 0.0, 0.0};
  }

  double2 ra0, ra1, rb0, rb1;
  // element i (0, 1) of this thread's share of a 64 x 16 stage
#define Z8_LDA(i, k0, dst)                                                             \
  do {                                                                                 \
    const int m_ = TA ? (tid >> 4) + 32 * (i) : (tid & 63);                           \
    const int k_ = TA ? (tid & 15) : (tid >> 6) + 8 * (i);                            \
    const int gm = m0 + m_, gk = (k0) + k_;                                            \
    dst = (gm < M && gk < K) ? (TA ? Ap[gk + int64_t(gm) * pr.lda]                    \
                                   : (SYMA && gm < gk) ? Ap[gk + int64_t(gm) * pr.lda]      \
                                                       : Ap[gm + int64_t(gk) * pr.lda])     \
                             : make_double2(0.0, 0.0);                                      \
  } while (0)
#define Z8_LDB(i, k0, dst)                                                             \
  do {                                                                                 \
    const int n_ = TB ? (tid & 63) : (tid >> 4) + 32 * (i);                           \
    const int k_ = TB ? (tid >> 6) + 8 * (i) : (tid & 15);                            \
    const int gn = n0 + n_, gk = (k0) + k_;                                            \
    dst = (gn < N && gk < K) ? (TB ? Bp[gn + int64_t(gk) * pr.ldb] : Bp[gk + int64_t(gn) * pr.ldb]) : make_double2(0.0, 0.0); \
  } while (0)
#define Z8_STA(buf, i, v) As[buf][TA ? (tid & 15) : (tid >> 6) + 8 * (i)][TA ? (tid >> 4) + 32 * (i) : (tid & 63)] = (v)
#define Z8_STB(buf, i, v) Bs[buf][TB ? (tid >> 6) + 8 * (i) : (tid & 15)][TB ? (tid & 63) : (tid >> 4) + 32 * (i)] = (v)
#define Z8_LOAD(k0)          \
  do {                       \
    Z8_LDA(0, k0, ra0);      \
    Z8_LDA(1, k0, ra1);      \
    Z8_LDB(0, k0, rb0);      \
    Z8_LDB(1, k0, rb1);      \
  } while (0)
#define Z8_STORE(buf)        \
  do {                       \
    Z8_STA(buf, 0, ra0);     \
    Z8_STA(buf, 1, ra1);     \
    Z8_STB(buf, 0, rb0);     \
    Z8_STB(buf, 1, rb1);     \
  } while (0)

  const int nk = (K + BK - 1) / BK;
  Z8_LOAD(0);
  Z8_STORE(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) Z8_LOAD((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      double2 av[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = As[cur][kr][wm * 32 + i * 16 + (lane & 15)];
      const double2 bv = Bs[cur][kr][wn * 16 + (lane & 15)];
      double as[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) as[i] = av[i].x + av[i].y;
      const double bs = bv.x + bv.y;
#pragma unroll
      for (int i = 0; i < 2; ++i) p1[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv.x, av[i].x, p1[i], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i) p2[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv.y, av[i].y, p2[i], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i) p3[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(bs, as[i], p3[i], 0, 0, 0);
    }
    if (kt + 1 < nk) Z8_STORE(cur ^ 1);
    __syncthreads();
  }
#undef Z8_LDA
#undef Z8_LDB
#undef Z8_STA
#undef Z8_STB
#undef Z8_LOAD
#undef Z8_STORE

  const double2* C0p = BETA ? C0 + pole * sC0 + pr.c0_off : EXTC0 ? C0 + pole * sC0 : nullptr;
  const ExtAddDesc xd = EXTC0 ? xe[pr.ext] : ExtAddDesc{};
  const XMap xm = EXTC0 ? stage_ext_maps<512>(&As[0][0][0], BM, pr, xd, xk, xi, m0, n0) : XMap{nullptr, 0, 0, 0};
  double2* Cp = C + pole * sC + pr.c_off;
#pragma unroll
  for (int i = 0; i < 2; ++i) {  // a chunk of four elements per 16-row block (eight spill with G_EXTC0)
    double2 v[4];
    int mm[4], nn[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      mm[r] = m0 + wm * 32 + i * 16 + (lane & 15);
      nn[r] = n0 + wn * 16 + F64_DROW(r, lane);
      v[r] = make_double2(p1[i][r] - p2[i][r], p3[i][r] - p1[i][r] - p2[i][r]);
    }
    store_chunk<FLAGS>(v, mm, nn, pr, C0p, Cp, xd, xk, xi, xm);
  }
}

// The same FP64 contraction for small problems: two waves per 32 x 32
// output tile, each a 32 x 16 half (two tiles per workgroup of four waves,
// the waves independent), operands read from global memory straight into the
// MFMA operand registers: no LDS and no barriers, so a tile whose problem is
// much smaller than 64 x 64 costs little.  K advances by 8 (two MFMA
// k-steps), all loads of a step issued before its products; an element
// outside the problem is read from the operand's first element and replaced
// by zero (no branches around loads).  A half holds a third of the
// accumulators of a whole tile, so that four waves fit a SIMD and hide one
// another's load latency; a half whose columns all lie beyond the problem
// exits at once.
template <int FLAGS>
__global__ __launch_bounds__(256, 4) void k_zgemm_w(const GemmProb* __restrict__ probs,
                                                 const TileRef* __restrict__ tiles, int64_t ntiles, int64_t npoles,
                                                 const double2* __restrict__ A, int64_t sA,
                                                 const double2* __restrict__ B, int64_t sB, const double2* C0,
                                                 int64_t sC0, double2* C, int64_t sC,
    const ExtAddDesc* __restrict__ xe, const ExtAddChild* __restrict__ xk, const int32_t* __restrict__ xi) {
  constexpr bool TA = (FLAGS & G_TA) != 0, TB = (FLAGS & G_TB) != 0;
  constexpr bool BETA = (FLAGS & G_BETA) != 0, EXTC0 = (FLAGS & G_EXTC0) != 0;
  constexpr bool SYMA = (FLAGS & G_SYMA) != 0, A32 = (FLAGS & G_A32) != 0;
  static_assert(!(SYMA && TA), "a lower-stored symmetric A is read untransposed");
  static_assert(!A32, "the FP64 kernels read FP64 operands");
  const int64_t total = ntiles * npoles;
  const int64_t wv = xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  const int64_t w = wv >> 1;
  if (w >= total) return;  // the whole wave; nothing here synchronises waves
  const int lane = threadIdx.x & 63;
  const int64_t pole = w / ntiles;
  const TileRef tr = tiles[w % ntiles];
  const GemmProb pr = probs[tr.prob];
  const int M = pr.m, N = pr.n, K = pr.k;
  const int m0 = tr.tm * 32, n0 = tr.tn * 32 + 16 * static_cast<int>(wv & 1);
  if (n0 >= N) return;  // the whole wave: no column of this half is in the problem
  const double2* Ap = A + pole * sA + pr.a_off;
  const double2* Bp = B + pole * sB + pr.b_off;
  const int r = lane & 15, kq = lane >> 4;

  d4 p1[2], p2[2], p3[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    p1[i] = d4{0.0, 0.0, 0.0, 0.0};
    p2[i] = d4{0.0, 0.0, 0.0, 0.0};
    p3[i] = d4{0.0, 0.0, 0.0, 0.0};
  }
  for (int k0 = 0; k0 < K; k0 += 8) {
    double2 a[2][2], b[2];
    bool oa[2][2], ob[2];
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      const int gk = k0 + 4 * st + kq;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int gm = m0 + 16 * i + r;
        oa[st][i] = gm < M && gk < K;
        const int64_t ia = (TA || (SYMA && gm < gk)) ? gk + int64_t(gm) * pr.lda : gm + int64_t(gk) * pr.lda;
        a[st][i] = Ap[oa[st][i] ? ia : int64_t(0)];
      }
      const int gn = n0 + r;
      ob[st] = gn < N && gk < K;
      const int64_t ib = TB ? gn + int64_t(gk) * pr.ldb : gk + int64_t(gn) * pr.ldb;
      b[st] = Bp[ob[st] ? ib : int64_t(0)];
    }
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      double ar[2], ai[2], as[2];
      const double br = ob[st] ? b[st].x : 0.0, bi = ob[st] ? b[st].y : 0.0, bs = br + bi;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ar[i] = oa[st][i] ? a[st][i].x : 0.0;
        ai[i] = oa[st][i] ? a[st][i].y : 0.0;
        as[i] = ar[i] + ai[i];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        p1[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(br, ar[i], p1[i], 0, 0, 0);
        p2[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(bi, ai[i], p2[i], 0, 0, 0);
        p3[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(bs, as[i], p3[i], 0, 0, 0);
      }
    }
  }

  const double2* C0p = BETA ? C0 + pole * sC0 + pr.c0_off : EXTC0 ? C0 + pole * sC0 : nullptr;
  const ExtAddDesc xd = EXTC0 ? xe[pr.ext] : ExtAddDesc{};
  const XMap xm{nullptr, 0, 0, 0};  // no LDS in this kernel: maps read from global memory
  double2* Cp = C + pole * sC + pr.c_off;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    double2 v[4];
    int mm[4], nn[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      mm[q] = m0 + i * 16 + (lane & 15);
      nn[q] = n0 + F64_DROW(q, lane);
      v[q] = make_double2(p1[i][q] - p2[i][q], p3[i][q] - p1[i][q] - p2[i][q]);
    }
    store_chunk<FLAGS>(v, mm, nn, pr, C0p, Cp, xd, xk, xi, xm);
  }
}

// Same contraction with the products on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32) and FP32 accumulation: FP64 operands are rounded
// to FP32 when staged into LDS, the four real products of each complex one
// are accumulated in FP32, and the result is formed in FP64 (scaled, added
// to C0 in FP64, stored as complex128).  Used for the front updates of poles
// away from the real axis.
typedef float f4 __attribute__((ext_vector_type(4)));

// WT x WT MFMA blocks of 16x16 per wave, NWR x NWR waves: the workgroup tile
// is (16 WT NWR) x (16 WT NWR).  WT = 2 on 2 x 2 waves gives the 64 x 64
// tiles; WT = 2 on 4 x 4 waves the 128 x 128 ones, four waves per SIMD with
// at most 128 registers each (4.4 % faster than WT = 4 on 2 x 2 waves, two
// per SIMD at 256 registers, with the same products in the same order).
template <int FLAGS, int WT, int NWR>
__global__ __launch_bounds__(64 * NWR * NWR, NWR == 2 ? 2 : 1) void k_cgemm32(const GemmProb* __restrict__ probs,
                                                    const TileRef* __restrict__ tiles, int64_t ntiles,
                                                    int64_t npoles, const double2* __restrict__ A, int64_t sA,
                                                    const double2* __restrict__ B, int64_t sB, const double2* C0,
                                                    int64_t sC0, double2* C, int64_t sC,
    const ExtAddDesc* __restrict__ xe, const ExtAddChild* __restrict__ xk, const int32_t* __restrict__ xi) {
  constexpr bool TA = (FLAGS & G_TA) != 0, TB = (FLAGS & G_TB) != 0, SYM = (FLAGS & G_SYM) != 0;
  constexpr bool BETA = (FLAGS & G_BETA) != 0, EXTC0 = (FLAGS & G_EXTC0) != 0;
  constexpr bool SYMA = (FLAGS & G_SYMA) != 0, A32 = (FLAGS & G_A32) != 0;
  static_assert(!(SYMA && TA), "a lower-stored symmetric A is read untransposed");
  constexpr int NT = 64 * NWR * NWR;   // threads
  constexpr int TM = 16 * WT * NWR;    // workgroup tile edge
  constexpr int NL = TM * BK / NT;     // operand elements per thread per stage
  constexpr int RS = NT / TM;          // k rows per pass of a non-transposed load
  constexpr int TR = NT / 16;          // rows per pass of a transposed load
  __shared__ float2 As[2][BK][TM + 1];
  __shared__ float2 Bs[2][BK][TM + 1];

  const int64_t total = ntiles * npoles;
  const int64_t logical = xcd_remap(blockIdx.x, total);
  const int64_t pole = logical / ntiles;
  const TileRef tr = tiles[logical % ntiles];
  const GemmProb pr = probs[tr.prob];
  const double2* Ap = A + pole * sA + pr.a_off;
  const double2* Bp = B + pole * sB + pr.b_off;
  const int M = pr.m, N = pr.n, K = pr.k;
  const int m0 = tr.tm * TM, n0 = tr.tn * TM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % NWR, wn = wave / NWR;

  f4 cre[WT][WT], cim[WT][WT];
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j) {
      cre[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      cim[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }

  // operand staging: NL elements per thread, kept in named registers through
  // a fully unrolled loop over a register array (no lambda captures, which
  // would move the array to scratch memory)
  double2 ra[NL], rb[NL];
#define CG_LOAD(k0)                                                                              \
  _Pragma("unroll") for (int i = 0; i < NL; ++i) {                                               \
    {                                                                                            \
      const int m_ = TA ? (tid >> 4) + TR * i : tid % TM;                                        \
      const int k_ = TA ? (tid & 15) : tid / TM + RS * i;                                        \
      const int gm = m0 + m_, gk = (k0) + k_;                                                    \
      ra[i] = (gm < M && gk < K)                                                                             \
                  ? (A32 ? ((SYMA && gm < gk) ? a_elem<true>(Ap, gk + int64_t(gm) * pr.lda)                 \
                                                  : a_elem<true>(Ap, gm + int64_t(gk) * pr.lda))             \
                         : TA ? Ap[gk + int64_t(gm) * pr.lda]                                                 \
                         : (SYMA && gm < gk) ? Ap[gk + int64_t(gm) * pr.lda]                                  \
                                             : Ap[gm + int64_t(gk) * pr.lda])                                 \
                                 : make_double2(0.0, 0.0);                                                   \
    }                                                                                            \
    {                                                                                            \
      const int n_ = TB ? tid % TM : (tid >> 4) + TR * i;                                        \
      const int k_ = TB ? tid / TM + RS * i : (tid & 15);                                        \
      const int gn = n0 + n_, gk = (k0) + k_;                                                    \
      rb[i] = (gn < N && gk < K) ? (TB ? Bp[gn + int64_t(gk) * pr.ldb] : Bp[gk + int64_t(gn) * pr.ldb]) : make_double2(0.0, 0.0); \
    }                                                                                            \
  }
#define CG_STORE(buf)                                                                                        \
  _Pragma("unroll") for (int i = 0; i < NL; ++i) {                                                           \
    As[buf][TA ? (tid & 15) : tid / TM + RS * i][TA ? (tid >> 4) + TR * i : tid % TM] =                    \
        make_float2(static_cast<float>(ra[i].x), static_cast<float>(ra[i].y));                               \
    Bs[buf][TB ? tid / TM + RS * i : (tid & 15)][TB ? tid % TM : (tid >> 4) + TR * i] =                    \
        make_float2(static_cast<float>(rb[i].x), static_cast<float>(rb[i].y));                               \
  }

  const int nk = (K + BK - 1) / BK;
  CG_LOAD(0)
  CG_STORE(0)
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      CG_LOAD((kt + 1) * BK)
    }
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      float2 av[WT], bv[WT];
#pragma unroll
      for (int i = 0; i < WT; ++i) {
        av[i] = As[cur][kr][wm * 16 * WT + i * 16 + (lane & 15)];
        bv[i] = Bs[cur][kr][wn * 16 * WT + i * 16 + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j) cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[j].x, av[i].x, cre[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j) cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[j].x, av[i].y, cim[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j) cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(-bv[j].y, av[i].y, cre[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j) cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[j].y, av[i].x, cim[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) {
      CG_STORE(cur ^ 1)
    }
    __syncthreads();
  }

  const double2* C0p = BETA ? C0 + pole * sC0 + pr.c0_off : EXTC0 ? C0 + pole * sC0 : nullptr;
  const ExtAddDesc xd = EXTC0 ? xe[pr.ext] : ExtAddDesc{};
  const XMap xm = EXTC0 ? stage_ext_maps<NT>(&As[0][0][0], TM, pr, xd, xk, xi, m0, n0) : XMap{nullptr, 0, 0, 0};
  double2* Cp = C + pole * sC + pr.c_off;
  // 16-column blocks per chunk: two hold too many registers within 128 (sixteen waves) or with the
  // epilogue's extend-add
  constexpr int CB = (NWR == 2 && !EXTC0) ? 2 : 1;
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j0 = 0; j0 < WT; j0 += CB) {
      double2 v[4 * CB];
      int mm[4 * CB], nn[4 * CB];
#pragma unroll
      for (int j = j0; j < j0 + CB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          mm[4 * (j - j0) + r] = m0 + wm * 16 * WT + i * 16 + (lane & 15);
          nn[4 * (j - j0) + r] = n0 + wn * 16 * WT + j * 16 + F32_DROW(r, lane);
          v[4 * (j - j0) + r] = make_double2(static_cast<double>(cre[i][j][r]), static_cast<double>(cim[i][j][r]));
        }
      store_chunk<FLAGS>(v, mm, nn, pr, C0p, Cp, xd, xk, xi, xm);
    }
}

// Same contraction with compensated split-BF16 products.  Operands are
// staged into LDS as FP32 (the only rounding of the operands, as in the FP32
// kernel); when a lane picks up its MFMA operand (8 consecutive k of one
// row) it splits every FP32 value x exactly into three bfloat16 numbers,
// x = h + m + l (h = bf16(x), m = bf16(x - h), l = x - h - m: 8 + 8 + 8
// significand bits, the differences exact in FP32), and the six products
// h.h, h.m, m.h, h.l, m.m, l.h of each real product run on the BF16 matrix
// cores (v_mfma_f32_16x16x32_bf16), which form bf16 x bf16 products exactly
// and accumulate in FP32.  The dropped products m.l, l.m, l.l are O(2^-24)
// relative, so the result has the accuracy of an FP32 GEMM for a quarter of
// its matrix-core cycles; the split runs on the vector ALUs beside them.
// TM x TM output tiles on NW waves in two rows: TM = 128 on eight waves
// (64 x 32 each), TM = 64 on four (32 x 32 each); K in steps of 32 through
// double-buffered LDS (re and im planes of FP32, rows padded to 36 floats so
// that the 16 rows read by one MFMA operand hit distinct banks).
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int B3_BK = 32;                // K per stage
constexpr int B3_LD = B3_BK + 4;         // LDS row stride (floats)

// exact split of 8 FP32 values into three bf16 vectors, two values per
// packed conversion (v_cvt_pk_bf16_f32 rounds to nearest even)
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 b2 __attribute__((ext_vector_type(2)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void split2(f2 x, unsigned& h, unsigned& m, unsigned& l) {
  const b2 hh = __builtin_convertvector(x, b2);
  const f2 r1 = x - __builtin_convertvector(hh, f2);
  const b2 mm = __builtin_convertvector(r1, b2);
  const f2 r2 = r1 - __builtin_convertvector(mm, f2);
  h = __builtin_bit_cast(unsigned, hh);
  m = __builtin_bit_cast(unsigned, mm);
  l = __builtin_bit_cast(unsigned, __builtin_convertvector(r2, b2));
}
__device__ __forceinline__ void split8(const f4& x0, const f4& x1, bf8& h, bf8& m, bf8& l) {
  unsigned h0, h1, h2, h3, m0, m1, m2, m3, l0, l1, l2, l3;
  split2(f2{x0[0], x0[1]}, h0, m0, l0);
  split2(f2{x0[2], x0[3]}, h1, m1, l1);
  split2(f2{x1[0], x1[1]}, h2, m2, l2);
  split2(f2{x1[2], x1[3]}, h3, m3, l3);
  h = __builtin_bit_cast(bf8, u4v{h0, h1, h2, h3});
  m = __builtin_bit_cast(bf8, u4v{m0, m1, m2, m3});
  l = __builtin_bit_cast(bf8, u4v{l0, l1, l2, l3});
}

template <int FLAGS, int B3_TM, int NW>
__global__ __launch_bounds__(NW * 64) void k_cgemm_bf3(const GemmProb* __restrict__ probs,
                                                   const TileRef* __restrict__ tiles, int64_t ntiles,
                                                   int64_t npoles, const double2* __restrict__ A, int64_t sA,
                                                   const double2* __restrict__ B, int64_t sB, const double2* C0,
                                                   int64_t sC0, double2* C, int64_t sC,
    const ExtAddDesc* __restrict__ xe, const ExtAddChild* __restrict__ xk, const int32_t* __restrict__ xi) {
  constexpr bool TA = (FLAGS & G_TA) != 0, TB = (FLAGS & G_TB) != 0, SYM = (FLAGS & G_SYM) != 0;
  constexpr bool BETA = (FLAGS & G_BETA) != 0, EXTC0 = (FLAGS & G_EXTC0) != 0;
  constexpr bool SYMA = (FLAGS & G_SYMA) != 0, A32 = (FLAGS & G_A32) != 0;
  static_assert(!(SYMA && TA), "a lower-stored symmetric A is read untransposed");
  constexpr int NT = NW * 64;              // threads
  constexpr int IB = B3_TM / 32;           // 16-row blocks of a wave's A rows (wave tile TM/2 x WCOL)
  constexpr int WCOL = 2 * B3_TM / NW;     // columns of a wave's tile
  constexpr int JB = WCOL / 16;            // 16-column blocks of a wave's B columns
  constexpr int GPT = B3_TM * 8 / NT;      // groups of 4 k per thread and operand in a stage
  constexpr int KGS = NT / B3_TM;          // k-group stride of a row-contiguous load
  constexpr int RPT = NT / 8;              // rows per pass of a k-contiguous load
  constexpr int B3_PLANE = B3_TM * B3_LD;  // floats per plane
  // [buffer][A re, A im, B re, B im][row][k]
  __shared__ __attribute__((aligned(16))) float lds[2][4 * B3_PLANE];

  const int64_t total = ntiles * npoles;
  const int64_t logical = xcd_remap(blockIdx.x, total);
  const int64_t pole = logical / ntiles;
  const TileRef tr = tiles[logical % ntiles];
  const GemmProb pr = probs[tr.prob];
  const double2* Ap = A + pole * sA + pr.a_off;
  const double2* Bp = B + pole * sB + pr.b_off;
  const int M = pr.m, N = pr.n, K = pr.k;
  const int m0 = tr.tm * B3_TM, n0 = tr.tn * B3_TM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;   // wave tile: rows TM/2 wm.., columns WCOL wn..

  f4 cre[IB][JB], cim[IB][JB];
#pragma unroll
  for (int i = 0; i < IB; ++i)
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      cre[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      cim[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }

  // Staging: each thread moves two groups of four consecutive k of one row
  // per operand.  Row-contiguous storage (A untransposed, B transposed) puts
  // consecutive threads on consecutive rows; k-contiguous storage (A
  // transposed, B untransposed) puts eight threads on the 32 k of a row.
  // The next stage goes through registers in two halves (A, then B) so that
  // fewer of them are held across the products.
  double2 rs[4 * GPT];
#define B3_AROW(g) (TA ? tid / 8 + RPT * (g) : tid % B3_TM)
#define B3_AK(g) (TA ? 4 * (tid % 8) : 4 * (tid / B3_TM + KGS * (g)))
#define B3_BROW(g) (TB ? tid % B3_TM : tid / 8 + RPT * (g))
#define B3_BK4(g) (TB ? 4 * (tid / B3_TM + KGS * (g)) : 4 * (tid % 8))
  // whole 128 x 32 blocks inside the matrix load without per-element guards
  const bool afull = m0 + B3_TM <= M, bfull = n0 + B3_TM <= N;
#define B3_AIDX(gm, gk) ((TA || (SYMA && (gm) < (gk))) ? (gk) + int64_t(gm) * pr.lda : (gm) + int64_t(gk) * pr.lda)
#define B3_BIDX(gn, gk) (TB ? (gn) + int64_t(gk) * pr.ldb : (gk) + int64_t(gn) * pr.ldb)
#define B3_LOADA(k0)                                                                                    \
  if (afull && (k0) + B3_BK <= K) {                                                                     \
    _Pragma("unroll") for (int g = 0; g < GPT; ++g)                                                     \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                                   \
        const int gm = m0 + B3_AROW(g), gk = (k0) + B3_AK(g) + q;                                       \
        rs[4 * g + q] = a_elem<A32>(Ap, B3_AIDX(gm, gk));                                               \
      }                                                                                                 \
  } else {                                                                                              \
    _Pragma("unroll") for (int g = 0; g < GPT; ++g)                                                     \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                                   \
        const int gm = m0 + B3_AROW(g), gk = (k0) + B3_AK(g) + q;                                       \
        rs[4 * g + q] = (gm < M && gk < K) ? a_elem<A32>(Ap, B3_AIDX(gm, gk)) : make_double2(0.0, 0.0); \
      }                                                                                                 \
  }
#define B3_LOADB(k0)                                                                                    \
  if (bfull && (k0) + B3_BK <= K) {                                                                     \
    _Pragma("unroll") for (int g = 0; g < GPT; ++g)                                                     \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                                   \
        const int gn = n0 + B3_BROW(g), gk = (k0) + B3_BK4(g) + q;                                      \
        rs[4 * g + q] = Bp[B3_BIDX(gn, gk)];                                                            \
      }                                                                                                 \
  } else {                                                                                              \
    _Pragma("unroll") for (int g = 0; g < GPT; ++g)                                                     \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                                   \
        const int gn = n0 + B3_BROW(g), gk = (k0) + B3_BK4(g) + q;                                      \
        rs[4 * g + q] = (gn < N && gk < K) ? Bp[B3_BIDX(gn, gk)] : make_double2(0.0, 0.0);              \
      }                                                                                                 \
  }
#define B3_PUT(buf, plane, row, kk, v)                                                                  \
  do {                                                                                                  \
    float* d_ = &lds[buf][(plane) * B3_PLANE + (row) * B3_LD + (kk)];                                   \
    *reinterpret_cast<f4*>(d_) = f4{static_cast<float>((v)[0].x), static_cast<float>((v)[1].x),          \
                                    static_cast<float>((v)[2].x), static_cast<float>((v)[3].x)};        \
    *reinterpret_cast<f4*>(d_ + B3_PLANE) = f4{static_cast<float>((v)[0].y), static_cast<float>((v)[1].y), \
                                               static_cast<float>((v)[2].y), static_cast<float>((v)[3].y)}; \
  } while (0)
#define B3_STOREA(buf) _Pragma("unroll") for (int g = 0; g < GPT; ++g) B3_PUT(buf, 0, B3_AROW(g), B3_AK(g), rs + 4 * g);
#define B3_STOREB(buf) _Pragma("unroll") for (int g = 0; g < GPT; ++g) B3_PUT(buf, 2, B3_BROW(g), B3_BK4(g), rs + 4 * g);

  const int nk = (K + B3_BK - 1) / B3_BK;
  B3_LOADA(0)
  B3_STOREA(0)
  B3_LOADB(0)
  B3_STOREB(0)
  __syncthreads();
  const int orow = lane & 15, ok = 8 * (lane >> 4);
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) {
      B3_LOADA((kt + 1) * B3_BK)
    }
    const float* L = lds[cur];
    bf8 b[JB][6];   // [j][2 slice + part]
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      const float* br = L + 2 * B3_PLANE + (wn * WCOL + j * 16 + orow) * B3_LD + ok;
      split8(*reinterpret_cast<const f4*>(br), *reinterpret_cast<const f4*>(br + 4), b[j][0], b[j][2], b[j][4]);
      split8(*reinterpret_cast<const f4*>(br + B3_PLANE), *reinterpret_cast<const f4*>(br + B3_PLANE + 4), b[j][1],
             b[j][3], b[j][5]);
    }
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      const float* ar = L + (wm * (B3_TM / 2) + i * 16 + orow) * B3_LD + ok;
      bf8 a[6], na[3];
      split8(*reinterpret_cast<const f4*>(ar), *reinterpret_cast<const f4*>(ar + 4), a[0], a[2], a[4]);
      split8(*reinterpret_cast<const f4*>(ar + B3_PLANE), *reinterpret_cast<const f4*>(ar + B3_PLANE + 4), a[1], a[3],
             a[5]);
#pragma unroll
      for (int sl = 0; sl < 3; ++sl) {  // -Im(A) slices: sign flip of the bf16 bits
        na[sl] = __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, a[2 * sl + 1]) ^ 0x80008000u);
      }
      // slice pairs (sa, sb) with sa + sb <= 2; re += Ar Br - Ai Bi,
      // im += Ai Br + Ar Bi (B tile as the first operand)
#pragma unroll
      for (int sa = 0; sa < 3; ++sa)
#pragma unroll
        for (int sb = 0; sb + sa < 3; ++sb) {
#pragma unroll
          for (int j = 0; j < JB; ++j)
            cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j][2 * sb], a[2 * sa], cre[i][j], 0, 0, 0);
#pragma unroll
          for (int j = 0; j < JB; ++j)
            cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j][2 * sb], a[2 * sa + 1], cim[i][j], 0, 0, 0);
#pragma unroll
          for (int j = 0; j < JB; ++j)
            cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j][2 * sb + 1], na[sa], cre[i][j], 0, 0, 0);
#pragma unroll
          for (int j = 0; j < JB; ++j)
            cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j][2 * sb + 1], a[2 * sa], cim[i][j], 0, 0, 0);
        }
      if (i == IB / 2 - 1 && more) {  // halfway: the next A block to LDS, fetch the next B block
        B3_STOREA(cur ^ 1)
        B3_LOADB((kt + 1) * B3_BK)
      }
    }
    if (more) {
      B3_STOREB(cur ^ 1)
    }
    __syncthreads();
  }
#undef B3_AROW
#undef B3_AK
#undef B3_BROW
#undef B3_BK4
#undef B3_AIDX
#undef B3_BIDX
#undef B3_LOADA
#undef B3_LOADB
#undef B3_PUT
#undef B3_STOREA
#undef B3_STOREB

  const double2* C0p = BETA ? C0 + pole * sC0 + pr.c0_off : EXTC0 ? C0 + pole * sC0 : nullptr;
  const ExtAddDesc xd = EXTC0 ? xe[pr.ext] : ExtAddDesc{};
  const XMap xm = EXTC0 ? stage_ext_maps<NT>(&lds[0][0], B3_TM, pr, xd, xk, xi, m0, n0) : XMap{nullptr, 0, 0, 0};
  double2* Cp = C + pole * sC + pr.c_off;
#pragma unroll
  for (int i = 0; i < IB; ++i) {
    double2 v[4 * JB];
    int mm[4 * JB], nn[4 * JB];
#pragma unroll
    for (int j = 0; j < JB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        mm[4 * j + r] = m0 + wm * (B3_TM / 2) + i * 16 + (lane & 15);
        nn[4 * j + r] = n0 + wn * WCOL + j * 16 + F32_DROW(r, lane);
        v[4 * j + r] = make_double2(static_cast<double>(cre[i][j][r]), static_cast<double>(cim[i][j][r]));
      }
    store_chunk<FLAGS>(v, mm, nn, pr, C0p, Cp, xd, xk, xi, xm);
  }
}

// Variant of k_cgemm_bf3 (128 x 128 tiles, eight waves of 64 x 32) that
// splits every element once per stage instead of once per wave that reads
// it: the next stage's FP64 values are fetched into registers while the
// matrix cores work, and between the two barriers of a step each thread
// rounds its share to FP32, splits it and stores the twelve bf16 planes
// (A and B, 3 slices x re/im; rows padded to 40 bf16) that the MFMA operands
// are read from directly.
constexpr int B3S_TM = 128;
constexpr int B3S_LD = B3_BK + 8;            // bf16 per plane row
constexpr int B3S_PLANE = B3S_TM * B3S_LD;   // bf16 per plane

template <int FLAGS>
__global__ __launch_bounds__(512) void k_cgemm_bf3s(const GemmProb* __restrict__ probs,
                                                    const TileRef* __restrict__ tiles, int64_t ntiles,
                                                    int64_t npoles, const double2* __restrict__ A, int64_t sA,
                                                    const double2* __restrict__ B, int64_t sB, const double2* C0,
                                                    int64_t sC0, double2* C, int64_t sC,
    const ExtAddDesc* __restrict__ xe, const ExtAddChild* __restrict__ xk, const int32_t* __restrict__ xi) {
  constexpr bool TA = (FLAGS & G_TA) != 0, TB = (FLAGS & G_TB) != 0, SYM = (FLAGS & G_SYM) != 0;
  constexpr bool BETA = (FLAGS & G_BETA) != 0, EXTC0 = (FLAGS & G_EXTC0) != 0;
  constexpr bool SYMA = (FLAGS & G_SYMA) != 0, A32 = (FLAGS & G_A32) != 0;
  static_assert(!(SYMA && TA), "a lower-stored symmetric A is read untransposed");
  // planes: [operand A/B][2 slice + part][row][k]
  __shared__ __attribute__((aligned(16))) unsigned short lds[12 * B3S_PLANE];

  const int64_t total = ntiles * npoles;
  const int64_t logical = xcd_remap(blockIdx.x, total);
  const int64_t pole = logical / ntiles;
  const TileRef tr = tiles[logical % ntiles];
  const GemmProb pr = probs[tr.prob];
  const double2* Ap = A + pole * sA + pr.a_off;
  const double2* Bp = B + pole * sB + pr.b_off;
  const int M = pr.m, N = pr.n, K = pr.k;
  const int m0 = tr.tm * B3S_TM, n0 = tr.tn * B3S_TM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;   // wave tile: rows 64 wm.., columns 32 wn..

  f4 cre[4][2], cim[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cre[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      cim[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }

  // staging map as in k_cgemm_bf3: two groups of four consecutive k of one
  // row per thread and operand
  double2 ra[8], rb[8];
  const bool afull = m0 + B3S_TM <= M, bfull = n0 + B3S_TM <= N;
#define S3_AROW(g) (TA ? tid / 8 + 64 * (g) : tid % 128)
#define S3_AK(g) (TA ? 4 * (tid % 8) : 4 * (tid / 128 + 4 * (g)))
#define S3_BROW(g) (TB ? tid % 128 : tid / 8 + 64 * (g))
#define S3_BK4(g) (TB ? 4 * (tid / 128 + 4 * (g)) : 4 * (tid % 8))
#define S3_AIDX(gm, gk) ((TA || (SYMA && (gm) < (gk))) ? (gk) + int64_t(gm) * pr.lda : (gm) + int64_t(gk) * pr.lda)
#define S3_BIDX(gn, gk) (TB ? (gn) + int64_t(gk) * pr.ldb : (gk) + int64_t(gn) * pr.ldb)
#define S3_LOAD(k0)                                                                                     \
  if (afull && (k0) + B3_BK <= K) {                                                                     \
    _Pragma("unroll") for (int g = 0; g < 2; ++g)                                                       \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                                   \
        const int gm = m0 + S3_AROW(g), gk = (k0) + S3_AK(g) + q;                                       \
        ra[4 * g + q] = a_elem<A32>(Ap, S3_AIDX(gm, gk));                                               \
      }                                                                                                 \
  } else {                                                                                              \
    _Pragma("unroll") for (int g = 0; g < 2; ++g)                                                       \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                                   \
        const int gm = m0 + S3_AROW(g), gk = (k0) + S3_AK(g) + q;                                       \
        ra[4 * g + q] = (gm < M && gk < K) ? a_elem<A32>(Ap, S3_AIDX(gm, gk)) : make_double2(0.0, 0.0); \
      }                                                                                                 \
  }                                                                                                     \
  if (bfull && (k0) + B3_BK <= K) {                                                                     \
    _Pragma("unroll") for (int g = 0; g < 2; ++g)                                                       \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                                   \
        const int gn = n0 + S3_BROW(g), gk = (k0) + S3_BK4(g) + q;                                      \
        rb[4 * g + q] = Bp[S3_BIDX(gn, gk)];                                                            \
      }                                                                                                 \
  } else {                                                                                              \
    _Pragma("unroll") for (int g = 0; g < 2; ++g)                                                       \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                                   \
        const int gn = n0 + S3_BROW(g), gk = (k0) + S3_BK4(g) + q;                                      \
        rb[4 * g + q] = (gn < N && gk < K) ? Bp[S3_BIDX(gn, gk)] : make_double2(0.0, 0.0);              \
      }                                                                                                 \
  }
  // split four complex values (one group) and store them into the six planes of an operand
#define S3_PUT(base, row, kk, v)                                                                        \
  do {                                                                                                  \
    unsigned h0, h1, m0_, m1, l0, l1;                                                                   \
    unsigned short* d_ = lds + (base) + (row) * B3S_LD + (kk);                                          \
    split2(f2{static_cast<float>((v)[0].x), static_cast<float>((v)[1].x)}, h0, m0_, l0);                \
    split2(f2{static_cast<float>((v)[2].x), static_cast<float>((v)[3].x)}, h1, m1, l1);                 \
    *reinterpret_cast<u2v*>(d_) = u2v{h0, h1};                                                          \
    *reinterpret_cast<u2v*>(d_ + 2 * B3S_PLANE) = u2v{m0_, m1};                                         \
    *reinterpret_cast<u2v*>(d_ + 4 * B3S_PLANE) = u2v{l0, l1};                                          \
    split2(f2{static_cast<float>((v)[0].y), static_cast<float>((v)[1].y)}, h0, m0_, l0);                \
    split2(f2{static_cast<float>((v)[2].y), static_cast<float>((v)[3].y)}, h1, m1, l1);                 \
    *reinterpret_cast<u2v*>(d_ + B3S_PLANE) = u2v{h0, h1};                                              \
    *reinterpret_cast<u2v*>(d_ + 3 * B3S_PLANE) = u2v{m0_, m1};                                         \
    *reinterpret_cast<u2v*>(d_ + 5 * B3S_PLANE) = u2v{l0, l1};                                          \
  } while (0)
#define S3_STORE()                                                                                      \
  _Pragma("unroll") for (int g = 0; g < 2; ++g) {                                                       \
    S3_PUT(0, S3_AROW(g), S3_AK(g), ra + 4 * g);                                                        \
    S3_PUT(6 * B3S_PLANE, S3_BROW(g), S3_BK4(g), rb + 4 * g);                                           \
  }

  const int nk = (K + B3_BK - 1) / B3_BK;
  S3_LOAD(0)
  S3_STORE()
  __syncthreads();
  const int orow = lane & 15, ok = 8 * (lane >> 4);
  for (int kt = 0; kt < nk; ++kt) {
    const bool more = kt + 1 < nk;
    if (more) {
      S3_LOAD((kt + 1) * B3_BK)
    }
    bf8 b[2][6];   // [j][2 slice + part]
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int pl = 0; pl < 6; ++pl)
        b[j][pl] = *reinterpret_cast<const bf8*>(lds + (6 + pl) * B3S_PLANE + (wn * 32 + j * 16 + orow) * B3S_LD + ok);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bf8 a[6], na[3];
#pragma unroll
      for (int pl = 0; pl < 6; ++pl)
        a[pl] = *reinterpret_cast<const bf8*>(lds + pl * B3S_PLANE + (wm * 64 + i * 16 + orow) * B3S_LD + ok);
#pragma unroll
      for (int sl = 0; sl < 3; ++sl)  // -Im(A) slices: sign flip of the bf16 bits
        na[sl] = __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, a[2 * sl + 1]) ^ 0x80008000u);
#pragma unroll
      for (int sa = 0; sa < 3; ++sa)
#pragma unroll
        for (int sb = 0; sb + sa < 3; ++sb) {
#pragma unroll
          for (int j = 0; j < 2; ++j)
            cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j][2 * sb], a[2 * sa], cre[i][j], 0, 0, 0);
#pragma unroll
          for (int j = 0; j < 2; ++j)
            cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j][2 * sb], a[2 * sa + 1], cim[i][j], 0, 0, 0);
#pragma unroll
          for (int j = 0; j < 2; ++j)
            cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j][2 * sb + 1], na[sa], cre[i][j], 0, 0, 0);
#pragma unroll
          for (int j = 0; j < 2; ++j)
            cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j][2 * sb + 1], a[2 * sa], cim[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
    if (more) {
      S3_STORE()
    }
    __syncthreads();
  }
#undef S3_AROW
#undef S3_AK
#undef S3_BROW
#undef S3_BK4
#undef S3_AIDX
#undef S3_BIDX
#undef S3_LOAD
#undef S3_PUT
#undef S3_STORE

  const double2* C0p = BETA ? C0 + pole * sC0 + pr.c0_off : EXTC0 ? C0 + pole * sC0 : nullptr;
  const ExtAddDesc xd = EXTC0 ? xe[pr.ext] : ExtAddDesc{};
  const XMap xm = EXTC0 ? stage_ext_maps<512>(lds, B3S_TM, pr, xd, xk, xi, m0, n0) : XMap{nullptr, 0, 0, 0};
  double2* Cp = C + pole * sC + pr.c_off;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double2 v[8];
    int mm[8], nn[8];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        mm[4 * j + r] = m0 + wm * 64 + i * 16 + (lane & 15);
        nn[4 * j + r] = n0 + wn * 32 + j * 16 + F32_DROW(r, lane);
        v[4 * j + r] = make_double2(static_cast<double>(cre[i][j][r]), static_cast<double>(cim[i][j][r]));
      }
    store_chunk<FLAGS>(v, mm, nn, pr, C0p, Cp, xd, xk, xi, xm);
  }
}

// Variant of the split-BF16 contraction that splits every operand element
// once, as it is staged, and never per wave: K advances 16 at a time, each
// stage holding the twelve bf16 planes of the A and B blocks (3 slices x
// re/im x 128 rows x 16 k, rows padded to 24 bf16), double-buffered in LDS,
// so that the next stage is fetched, rounded to FP32, split and stored while
// the matrix cores work on the current one, with one barrier per stage.  The
// products run on v_mfma_f32_32x32x16_bf16 (the 16-k bf16 shape at full rate
// on this matrix core): eight waves, each a 64 x 32 piece of the 128 x 128
// tile as two 32 x 32 blocks.
typedef float f16v __attribute__((ext_vector_type(16)));
constexpr int B3P_TM = 128;                  // tile edge
constexpr int B3P_BK = 16;                   // K per stage
constexpr int B3P_LD = B3P_BK + 8;           // bf16 per plane row
constexpr int B3P_PLANE = B3P_TM * B3P_LD;   // bf16 per plane
constexpr int B3P_STAGE = 12 * B3P_PLANE;    // A planes 0..5, B planes 6..11
constexpr uint32_t B3P_OOB = 0x7FFFFFF0u;    // descriptor range in bytes; offsets at or beyond it read zero

template <int FLAGS>
__global__ __launch_bounds__(512) void k_cgemm_bf3p(const GemmProb* __restrict__ probs,
                                                    const TileRef* __restrict__ tiles, int64_t ntiles,
                                                    int64_t npoles, const double2* __restrict__ A, int64_t sA,
                                                    const double2* __restrict__ B, int64_t sB, const double2* C0,
                                                    int64_t sC0, double2* C, int64_t sC,
    const ExtAddDesc* __restrict__ xe, const ExtAddChild* __restrict__ xk, const int32_t* __restrict__ xi) {
  constexpr bool TA = (FLAGS & G_TA) != 0, TB = (FLAGS & G_TB) != 0, SYM = (FLAGS & G_SYM) != 0;
  constexpr bool BETA = (FLAGS & G_BETA) != 0, EXTC0 = (FLAGS & G_EXTC0) != 0;
  constexpr bool SYMA = (FLAGS & G_SYMA) != 0, A32 = (FLAGS & G_A32) != 0;
  static_assert(!(SYMA && TA), "a lower-stored symmetric A is read untransposed");
  // [stage][plane = 6 operand + 2 slice + part][row][k]
  __shared__ __attribute__((aligned(16))) unsigned short lds[2 * B3P_STAGE];

  const int64_t total = ntiles * npoles;
  const int64_t logical = xcd_remap(blockIdx.x, total);
  const int64_t pole = logical / ntiles;
  const TileRef tr = tiles[logical % ntiles];
  const GemmProb pr = probs[tr.prob];
  const double2* Ap = A + pole * sA + pr.a_off;
  const double2* Bp = B + pole * sB + pr.b_off;
  const int M = pr.m, N = pr.n, K = pr.k;
  const int m0 = tr.tm * B3P_TM, n0 = tr.tn * B3P_TM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;   // wave piece: rows 64 wm.., columns 32 wn..

  f16v cre[2], cim[2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      cre[i][r] = 0.f;
      cim[i][r] = 0.f;
    }

  // Staging: every thread moves four consecutive k of one row per operand
  // and stage.  Row-contiguous storage (A untransposed, B transposed) puts
  // consecutive threads on consecutive rows; k-contiguous storage puts four
  // threads on the 16 k of a row.
  const int arow = TA ? tid / 4 : tid % B3P_TM, ak = TA ? 4 * (tid % 4) : 4 * (tid / B3P_TM);
  const int brow = TB ? tid % B3P_TM : tid / 4, bk = TB ? 4 * (tid / B3P_TM) : 4 * (tid % 4);
  double2 ra0[4], rb0[4], ra1[4], rb1[4];   // two stages in flight
  // Branch-free fetches through buffer descriptors: an element outside the
  // problem gets an offset beyond the descriptor's range, which the hardware
  // answers with zeros, so no load is guarded by a branch and the waits for
  // one stage's loads do not cover the next stage's.  Byte offsets are
  // 32-bit: every operand region of a problem spans less than B3P_OOB bytes
  // (the launcher checks this before choosing the kernel).
  const __amdgpu_buffer_rsrc_t arsrc =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double2*>(Ap), static_cast<short>(0), B3P_OOB, 0x00020000);
  const __amdgpu_buffer_rsrc_t brsrc =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double2*>(Bp), static_cast<short>(0), B3P_OOB, 0x00020000);
  const uint32_t ulda = static_cast<uint32_t>(pr.lda), uldb = static_cast<uint32_t>(pr.ldb);
  const uint32_t gm = static_cast<uint32_t>(m0 + arow), gn = static_cast<uint32_t>(n0 + brow);
  const uint32_t uM = static_cast<uint32_t>(M), uN = static_cast<uint32_t>(N), uK = static_cast<uint32_t>(K);
#define P3_LOAD(k0, ra, rb)                                                                             \
  {                                                                                                     \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                                     \
      const uint32_t gk = static_cast<uint32_t>((k0) + ak + q);                                         \
      const uint32_t o = (TA || (SYMA && gm < gk)) ? gk + gm * ulda : gm + gk * ulda;                   \
      if (A32) {                                                                                        \
        const float2 x_ = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(               \
                                              arsrc, (gm < uM && gk < uK) ? o * 8u : B3P_OOB, 0, 0));   \
        ra[q] = make_double2(static_cast<double>(x_.x), static_cast<double>(x_.y));                     \
      } else {                                                                                          \
        ra[q] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(                      \
                                                arsrc, (gm < uM && gk < uK) ? o * 16u : B3P_OOB, 0, 0)); \
      }                                                                                                 \
    }                                                                                                   \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                                     \
      const uint32_t gk = static_cast<uint32_t>((k0) + bk + q);                                         \
      const uint32_t o = TB ? gn + gk * uldb : gk + gn * uldb;                                          \
      rb[q] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(                        \
                                              brsrc, (gn < uN && gk < uK) ? o * 16u : B3P_OOB, 0, 0));  \
    }                                                                                                   \
  }
  // round four complex values to FP32, split them and store the six planes of one operand row
#define P3_PUT(base, row, kk, v)                                                                        \
  do {                                                                                                  \
    unsigned h0, h1, m0_, m1, l0, l1;                                                                   \
    unsigned short* d_ = lds + (base) + (row) * B3P_LD + (kk);                                          \
    split2(f2{static_cast<float>((v)[0].x), static_cast<float>((v)[1].x)}, h0, m0_, l0);                \
    split2(f2{static_cast<float>((v)[2].x), static_cast<float>((v)[3].x)}, h1, m1, l1);                 \
    *reinterpret_cast<u2v*>(d_) = u2v{h0, h1};                                                          \
    *reinterpret_cast<u2v*>(d_ + 2 * B3P_PLANE) = u2v{m0_, m1};                                         \
    *reinterpret_cast<u2v*>(d_ + 4 * B3P_PLANE) = u2v{l0, l1};                                          \
    split2(f2{static_cast<float>((v)[0].y), static_cast<float>((v)[1].y)}, h0, m0_, l0);                \
    split2(f2{static_cast<float>((v)[2].y), static_cast<float>((v)[3].y)}, h1, m1, l1);                 \
    *reinterpret_cast<u2v*>(d_ + B3P_PLANE) = u2v{h0, h1};                                              \
    *reinterpret_cast<u2v*>(d_ + 3 * B3P_PLANE) = u2v{m0_, m1};                                         \
    *reinterpret_cast<u2v*>(d_ + 5 * B3P_PLANE) = u2v{l0, l1};                                          \
  } while (0)
#define P3_STORE(stage, ra, rb)                                                                         \
  {                                                                                                     \
    /* the fetched values enter the split here and not earlier, so that their */                       \
    /* wait is placed here, a whole stage after the fetch */                                            \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                                     \
      asm volatile("" : "+v"(ra[q].x), "+v"(ra[q].y), "+v"(rb[q].x), "+v"(rb[q].y));                   \
    }                                                                                                   \
    P3_PUT((stage) * B3P_STAGE, arow, ak, ra);                                                          \
    P3_PUT((stage) * B3P_STAGE + 6 * B3P_PLANE, brow, bk, rb);                                          \
  }

  // Stage kt + 2 is fetched while stage kt is multiplied and stage kt + 1
  // (fetched one step earlier) is split into the other LDS buffer.  The loop
  // is unrolled by two so that the two register sets keep fixed names, and
  // its body has no branch: the stage count is rounded up to even and the
  // fetches past K read zeros, so the compiler's wait for one stage's loads
  // leaves the next stage's in flight.
  const int nk = (K + B3P_BK - 1) / B3P_BK, nk2 = nk + (nk & 1);
  P3_LOAD(0, ra0, rb0)
  P3_STORE(0, ra0, rb0)
  P3_LOAD(B3P_BK, ra1, rb1)
  __syncthreads();
  // MFMA operand of lane l: row l % 32 of its 32-row block, k = 8 (l / 32) .. + 7
  const int orow = lane & 31, ok = 8 * (lane >> 5);
#define P3_STEP(kt, rnow, bnow, rnext, bnext)                                                           \
  {                                                                                                     \
    P3_LOAD(((kt) + 2) * B3P_BK, rnow, bnow)                                                            \
    asm volatile("" ::: "memory"); /* keeps the fetches here, ahead of their use */                     \
    P3_MMA((kt) & 1)                                                                                    \
    P3_STORE(((kt) & 1) ^ 1, rnext, bnext)                                                              \
    __syncthreads();                                                                                    \
  }
#define P3_MMA(cur)                                                                                     \
  {                                                                                                     \
    const unsigned short* L = lds + (cur) * B3P_STAGE;                                                  \
    bf8 b[6];                                                                                           \
    _Pragma("unroll") for (int pl = 0; pl < 6; ++pl)                                                    \
      b[pl] = *reinterpret_cast<const bf8*>(L + (6 + pl) * B3P_PLANE + (wn * 32 + orow) * B3P_LD + ok); \
    _Pragma("unroll") for (int i = 0; i < 2; ++i) {                                                     \
      bf8 a[6], na[3];                                                                                  \
      _Pragma("unroll") for (int pl = 0; pl < 6; ++pl)                                                  \
        a[pl] = *reinterpret_cast<const bf8*>(L + pl * B3P_PLANE + (wm * 64 + i * 32 + orow) * B3P_LD + ok); \
      _Pragma("unroll") for (int sl = 0; sl < 3; ++sl)                                                  \
        na[sl] = __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, a[2 * sl + 1]) ^ 0x80008000u);         \
      _Pragma("unroll") for (int sa = 0; sa < 3; ++sa)                                                  \
        _Pragma("unroll") for (int sb = 0; sb + sa < 3; ++sb) {                                         \
          cre[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[2 * sb], a[2 * sa], cre[i], 0, 0, 0);      \
          cim[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[2 * sb], a[2 * sa + 1], cim[i], 0, 0, 0);  \
          cre[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[2 * sb + 1], na[sa], cre[i], 0, 0, 0);     \
          cim[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[2 * sb + 1], a[2 * sa], cim[i], 0, 0, 0);  \
        }                                                                                               \
    }                                                                                                   \
  }
  // -Im(A) slices by a sign flip of the bf16 bits; slice pairs (sa, sb) with
  // sa + sb <= 2; re += Ar Br - Ai Bi, im += Ai Br + Ar Bi (B block first)
  for (int kt = 0; kt < nk2; kt += 2) {
    P3_STEP(kt, ra0, rb0, ra1, rb1)
    P3_STEP(kt + 1, ra1, rb1, ra0, rb0)
  }
#undef P3_STEP
#undef P3_MMA
#undef P3_LOAD
#undef P3_PUT
#undef P3_STORE

  // accumulator register r of lane l holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]:
  // row = column n of the tile (B block first), column = row m
  const double2* C0p = BETA ? C0 + pole * sC0 + pr.c0_off : EXTC0 ? C0 + pole * sC0 : nullptr;
  const ExtAddDesc xd = EXTC0 ? xe[pr.ext] : ExtAddDesc{};
  const XMap xm = EXTC0 ? stage_ext_maps<512>(lds, B3P_TM, pr, xd, xk, xi, m0, n0) : XMap{nullptr, 0, 0, 0};
  double2* Cp = C + pole * sC + pr.c_off;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // chunks of eight registers
      double2 v[8];
      int mm[8], nn[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int r = 8 * h + t;
        mm[t] = m0 + wm * 64 + i * 32 + (lane & 31);
        nn[t] = n0 + wn * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        v[t] = make_double2(static_cast<double>(cre[i][r]), static_cast<double>(cim[i][r]));
      }
      store_chunk<FLAGS>(v, mm, nn, pr, C0p, Cp, xd, xk, xi, xm);
    }
}

// Sixteen-wave form of the pre-split contraction: the same 128 x 128 tile,
// the same twelve bf16 planes per 16-k stage in LDS (double-buffered) and the
// same slice products in the same order per accumulator (so the results are
// those of k_cgemm_bf3p bit for bit), but each wave computes one 32 x 32
// block, four waves per SIMD.  Each thread stages two consecutive k of one
// row per operand and stage.
template <int FLAGS>
__global__ __launch_bounds__(1024) void k_cgemm_bf3w(const GemmProb* __restrict__ probs,
                                                    const TileRef* __restrict__ tiles, int64_t ntiles,
                                                    int64_t npoles, const double2* __restrict__ A, int64_t sA,
                                                    const double2* __restrict__ B, int64_t sB, const double2* C0,
                                                    int64_t sC0, double2* C, int64_t sC,
    const ExtAddDesc* __restrict__ xe, const ExtAddChild* __restrict__ xk, const int32_t* __restrict__ xi) {
  constexpr bool TA = (FLAGS & G_TA) != 0, TB = (FLAGS & G_TB) != 0;
  constexpr bool BETA = (FLAGS & G_BETA) != 0, EXTC0 = (FLAGS & G_EXTC0) != 0;
  constexpr bool SYMA = (FLAGS & G_SYMA) != 0, A32 = (FLAGS & G_A32) != 0;
  static_assert(!(SYMA && TA), "a lower-stored symmetric A is read untransposed");
  __shared__ __attribute__((aligned(16))) unsigned short lds[2 * B3P_STAGE];

  const int64_t total = ntiles * npoles;
  const int64_t logical = xcd_remap(blockIdx.x, total);
  const int64_t pole = logical / ntiles;
  const TileRef tr = tiles[logical % ntiles];
  const GemmProb pr = probs[tr.prob];
  const double2* Ap = A + pole * sA + pr.a_off;
  const double2* Bp = B + pole * sB + pr.b_off;
  const int M = pr.m, N = pr.n, K = pr.k;
  const int m0 = tr.tm * B3P_TM, n0 = tr.tn * B3P_TM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 3, wn = wave >> 2;   // wave block: rows 32 wm.., columns 32 wn..

  f16v cre, cim;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    cre[r] = 0.f;
    cim[r] = 0.f;
  }

  // staging position: each half-wave covers 8 consecutive rows x 4 pairs of
  // k, so that its 4-byte stores of one plane (rows 12 banks apart) hit 32
  // distinct banks (the store pass of 32 lanes over 32 banks)
  const int srow = 16 * (wave & 7) + (lane & 7) + 8 * (lane >> 5), sk = 2 * (((lane >> 3) & 3) + 4 * (wave >> 3));
  const int arow = srow, ak = sk, brow = srow, bk = sk;
  double2 ra0[2], rb0[2], ra1[2], rb1[2];   // two stages in flight
  const __amdgpu_buffer_rsrc_t arsrc =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double2*>(Ap), static_cast<short>(0), B3P_OOB, 0x00020000);
  const __amdgpu_buffer_rsrc_t brsrc =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double2*>(Bp), static_cast<short>(0), B3P_OOB, 0x00020000);
  const uint32_t ulda = static_cast<uint32_t>(pr.lda), uldb = static_cast<uint32_t>(pr.ldb);
  const uint32_t gm = static_cast<uint32_t>(m0 + arow), gn = static_cast<uint32_t>(n0 + brow);
  const uint32_t uM = static_cast<uint32_t>(M), uN = static_cast<uint32_t>(N), uK = static_cast<uint32_t>(K);
#define W3_LOAD(k0, ra, rb)                                                                             \
  {                                                                                                     \
    _Pragma("unroll") for (int q = 0; q < 2; ++q) {                                                     \
      const uint32_t gk = static_cast<uint32_t>((k0) + ak + q);                                         \
      const uint32_t o = (TA || (SYMA && gm < gk)) ? gk + gm * ulda : gm + gk * ulda;                   \
      if (A32) {                                                                                        \
        const float2 x_ = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(               \
                                              arsrc, (gm < uM && gk < uK) ? o * 8u : B3P_OOB, 0, 0));   \
        ra[q] = make_double2(static_cast<double>(x_.x), static_cast<double>(x_.y));                     \
      } else {                                                                                          \
        ra[q] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(                      \
                                                arsrc, (gm < uM && gk < uK) ? o * 16u : B3P_OOB, 0, 0)); \
      }                                                                                                 \
    }                                                                                                   \
    _Pragma("unroll") for (int q = 0; q < 2; ++q) {                                                     \
      const uint32_t gk = static_cast<uint32_t>((k0) + bk + q);                                         \
      const uint32_t o = TB ? gn + gk * uldb : gk + gn * uldb;                                          \
      rb[q] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(                        \
                                              brsrc, (gn < uN && gk < uK) ? o * 16u : B3P_OOB, 0, 0));  \
    }                                                                                                   \
  }
#define W3_PUT(base, row, kk, v)                                                                        \
  do {                                                                                                  \
    unsigned h_, m_, l_;                                                                                \
    unsigned short* d_ = lds + (base) + (row) * B3P_LD + (kk);                                          \
    split2(f2{static_cast<float>((v)[0].x), static_cast<float>((v)[1].x)}, h_, m_, l_);                 \
    *reinterpret_cast<unsigned*>(d_) = h_;                                                              \
    *reinterpret_cast<unsigned*>(d_ + 2 * B3P_PLANE) = m_;                                              \
    *reinterpret_cast<unsigned*>(d_ + 4 * B3P_PLANE) = l_;                                              \
    split2(f2{static_cast<float>((v)[0].y), static_cast<float>((v)[1].y)}, h_, m_, l_);                 \
    *reinterpret_cast<unsigned*>(d_ + B3P_PLANE) = h_;                                                  \
    *reinterpret_cast<unsigned*>(d_ + 3 * B3P_PLANE) = m_;                                              \
    *reinterpret_cast<unsigned*>(d_ + 5 * B3P_PLANE) = l_;                                              \
  } while (0)
#define W3_STORE(stage, ra, rb)                                                                         \
  {                                                                                                     \
    _Pragma("unroll") for (int q = 0; q < 2; ++q) {                                                     \
      asm volatile("" : "+v"(ra[q].x), "+v"(ra[q].y), "+v"(rb[q].x), "+v"(rb[q].y));                   \
    }                                                                                                   \
    W3_PUT((stage) * B3P_STAGE, arow, ak, ra);                                                          \
    W3_PUT((stage) * B3P_STAGE + 6 * B3P_PLANE, brow, bk, rb);                                          \
  }

  const int nk = (K + B3P_BK - 1) / B3P_BK, nk2 = nk + (nk & 1);
  W3_LOAD(0, ra0, rb0)
  W3_STORE(0, ra0, rb0)
  W3_LOAD(B3P_BK, ra1, rb1)
  __syncthreads();
  const int orow = lane & 31, ok = 8 * (lane >> 5);
#define W3_STEP(kt, rnow, bnow, rnext, bnext)                                                           \
  {                                                                                                     \
    W3_LOAD(((kt) + 2) * B3P_BK, rnow, bnow)                                                            \
    asm volatile("" ::: "memory");                                                                      \
    W3_MMA((kt) & 1)                                                                                    \
    W3_STORE(((kt) & 1) ^ 1, rnext, bnext)                                                              \
    __syncthreads();                                                                                    \
  }
#define W3_MMA(cur)                                                                                     \
  {                                                                                                     \
    const unsigned short* L = lds + (cur) * B3P_STAGE;                                                  \
    bf8 a[6], b[6], na[3];                                                                              \
    _Pragma("unroll") for (int pl = 0; pl < 6; ++pl)                                                    \
      b[pl] = *reinterpret_cast<const bf8*>(L + (6 + pl) * B3P_PLANE + (wn * 32 + orow) * B3P_LD + ok); \
    _Pragma("unroll") for (int pl = 0; pl < 6; ++pl)                                                    \
      a[pl] = *reinterpret_cast<const bf8*>(L + pl * B3P_PLANE + (wm * 32 + orow) * B3P_LD + ok);       \
    _Pragma("unroll") for (int sl = 0; sl < 3; ++sl)                                                    \
      na[sl] = __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, a[2 * sl + 1]) ^ 0x80008000u);           \
    _Pragma("unroll") for (int sa = 0; sa < 3; ++sa)                                                    \
      _Pragma("unroll") for (int sb = 0; sb + sa < 3; ++sb) {                                           \
        cre = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[2 * sb], a[2 * sa], cre, 0, 0, 0);              \
        cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[2 * sb], a[2 * sa + 1], cim, 0, 0, 0);          \
        cre = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[2 * sb + 1], na[sa], cre, 0, 0, 0);             \
        cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[2 * sb + 1], a[2 * sa], cim, 0, 0, 0);          \
      }                                                                                                 \
  }
  for (int kt = 0; kt < nk2; kt += 2) {
    W3_STEP(kt, ra0, rb0, ra1, rb1)
    W3_STEP(kt + 1, ra1, rb1, ra0, rb0)
  }
#undef W3_STEP
#undef W3_MMA
#undef W3_LOAD
#undef W3_PUT
#undef W3_STORE

  const double2* C0p = BETA ? C0 + pole * sC0 + pr.c0_off : EXTC0 ? C0 + pole * sC0 : nullptr;
  const ExtAddDesc xd = EXTC0 ? xe[pr.ext] : ExtAddDesc{};
  const XMap xm = EXTC0 ? stage_ext_maps<1024>(lds, B3P_TM, pr, xd, xk, xi, m0, n0) : XMap{nullptr, 0, 0, 0};
  double2* Cp = C + pole * sC + pr.c_off;
#pragma unroll
  for (int h = 0; h < 4; ++h) {  // chunks of four registers (eight spill with G_EXTC0)
    double2 v[4];
    int mm[4], nn[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int r = 4 * h + t;
      mm[t] = m0 + wm * 32 + (lane & 31);
      nn[t] = n0 + wn * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      v[t] = make_double2(static_cast<double>(cre[r]), static_cast<double>(cim[r]));
    }
    store_chunk<FLAGS>(v, mm, nn, pr, C0p, Cp, xd, xk, xi, xm);
  }
}

// ----------------------------------------------------------------- copy
//
// dst (rows x cols) <- src, or <- src^T through an LDS tile so that both the
// reads and the writes run down columns.
template <bool TRANS>
__global__ __launch_bounds__(256) void k_copy(const CopyDesc* __restrict__ descs, const CopyTile* __restrict__ tiles,
                                              const double2* __restrict__ src, int64_t ss, double2* __restrict__ dst,
                                              int64_t ds) {
  __shared__ double2 t[64][65];
  const CopyTile ct = tiles[blockIdx.x];
  const CopyDesc d = descs[ct.desc];
  const double2* s = src + int64_t(blockIdx.y) * ss + d.src_off;
  double2* o = dst + int64_t(blockIdx.y) * ds + d.dst_off;
  const int tid = threadIdx.x;
  if (!TRANS) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int r = ct.r0 + (tid & 63), c = ct.c0 + (tid >> 6) + 4 * i;
      if (r < d.rows && c < d.cols) o[r + int64_t(c) * d.ldd] = s[r + int64_t(c) * d.lds];
    }
  } else {
    // dst(r, c) = src(c, r): read src rows c0.. (as its row index) coalesced
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int sr = tid & 63, sc = (tid >> 6) + 4 * i;  // src row = dst col, src col = dst row
      const int gr = ct.c0 + sr, gc = ct.r0 + sc;
      if (gr < d.cols && gc < d.rows) t[sc][sr] = s[gr + int64_t(gc) * d.lds];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int r = tid & 63, c = (tid >> 6) + 4 * i;
      const int gr = ct.r0 + r, gc = ct.c0 + c;
      if (gr < d.rows && gc < d.cols) o[gr + int64_t(gc) * d.ldd] = t[r][c];
    }
  }
}

// ----------------------------------------------------------------- gather G_UU
//
// Downward pass: the lower triangle of G on U_f x U_f is read from the
// parent's selected block, i.e. from its G_JJ and G_UJ panel or from the
// parent's own gathered G_UU (Eq. (38): the blocks X^{-1}_{p,2n},
// X^{-1}_{p,2n+1} needed by the next level).
__global__ __launch_bounds__(256) void k_gather(const GatherDesc* __restrict__ descs,
                                                const int32_t* __restrict__ rel, const ElemTile* __restrict__ tiles,
                                                const double2* __restrict__ pguu, int64_t gs,
                                                const double2* __restrict__ panel, int64_t ps,
                                                double2* __restrict__ guu, int64_t us, int64_t nhi, int in32,
                                                int out32) {
  const int64_t pole = blockIdx.y;
  // poles from nhi on: the parent's G_UU is FP32 complex (in32), and so is
  // the output (out32) when its only consumer, G_UJ = -G_UU L, runs in low
  // precision (it rounds the operand to FP32 in any case)
  const bool lo = pole >= nhi, rd32 = lo && in32 != 0, wr32 = lo && out32 != 0;
  const ElemTile t = tiles[blockIdx.x];
  const GatherDesc d = descs[t.desc];
  const uint32_t total = uint32_t(d.nu) * d.nu;
  const int32_t* rl = rel + d.rel_off;
  const double2* pan = panel + pole * ps + d.ppanel_off;
  const double2* pg = pguu + pole * gs + d.pguu_off;
  double2* out = guu + pole * us + d.dst_off;
  const int64_t pld = d.pnj + d.pnu;
  // four elements per thread: the map reads of all four, then their value
  // reads, are in flight together
  uint32_t e[4];
  bool live[4];
  int r[4], s[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    e[i] = uint32_t(t.e0) + threadIdx.x + 256 * i;
    const uint32_t b = e[i] / uint32_t(d.nu), a = e[i] - b * uint32_t(d.nu);
    live[i] = e[i] < total && a >= b;  // G_UU is kept as its lower triangle
    r[i] = live[i] ? rl[a] : 0;
    s[i] = live[i] ? rl[b] : 0;  // r >= s (increasing map)
  }
  double2 v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t gi = (r[i] - d.pnj) + int64_t(s[i] - d.pnj) * d.pnu;
    v[i] = !live[i] ? make_double2(0.0, 0.0)
           : s[i] < d.pnj ? pan[r[i] + int64_t(s[i]) * pld]
           : rd32 ? a_elem<true>(pg, gi) : pg[gi];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (!live[i]) continue;
    if (wr32)
      reinterpret_cast<float2*>(out)[e[i]] = make_float2(static_cast<float>(v[i].x), static_cast<float>(v[i].y));
    else
      out[e[i]] = v[i];
  }
}

// ----------------------------------------------------------------- pole sum
//
// acc[k] += sum_p w_p Re G_p[slot_k], poles in increasing order (Eq. (8)):
// one thread per pattern position, positions sorted by panel offset so that
// a wave reads neighbouring panel entries.
__global__ __launch_bounds__(256) void k_accum(const int64_t* __restrict__ slot, int64_t count,
                                               const double2* __restrict__ panel, int64_t ps,
                                               const double* __restrict__ w, int npoles, double* __restrict__ acc) {
  const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (k >= count) return;
  const double* pr = reinterpret_cast<const double*>(panel) + 2 * slot[k];
  double v = acc[k];
  for (int p = 0; p < npoles; ++p) v += w[p] * pr[2 * int64_t(p) * ps];
  acc[k] = v;
}

// Starts the sum at M0 (or 0) and clears the pivot status words (a kernel
// rather than a memset, so the sequence can be captured in a graph).
__global__ __launch_bounds__(256) void k_init_acc(const double* __restrict__ m0, int64_t count, int add_m0,
                                                  double* __restrict__ acc, int* __restrict__ status) {
  const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (k < 4) status[k] = 0;
  if (k < count) acc[k] = add_m0 ? m0[k] : 0.0;
}

__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ entry, int64_t count,
                                                 const double* __restrict__ acc, double* __restrict__ out) {
  const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (k < count) out[entry[k]] = acc[k];
}

// Plain streaming copy (16-byte elements), the calibration reference for
// HBM byte counters.
__global__ __launch_bounds__(256) void k_stream_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                                                     int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) dst[i] = src[i];
}

// ----------------------------------------------------------------- launchers

hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, hipStream_t st) {
  const int64_t n = bytes / 16;
  if (n == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 256 * 64);
  hipLaunchKernelGGL(k_stream_copy, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                     static_cast<const double2*>(src), static_cast<double2*>(dst), n);
  return hipGetLastError();
}

static inline unsigned blocks_for(int64_t n, int per) { return static_cast<unsigned>((n + per - 1) / per); }

hipError_t launch_extadd(const DevOp& o, hipStream_t st) {
  if (o.tile_count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_extadd, dim3(static_cast<unsigned>(o.tile_count), o.npoles), dim3(256), 0, st, o.ext, o.ext_child,
                     o.ext_inv, o.elem_tiles, o.tile_count, o.c, o.sc, o.a, o.sa);
  return hipGetLastError();
}

hipError_t launch_assemble(const DevOp& o, const double* hv, const double* sv, const double2* alpha,
                           int64_t astride, double hcoef, hipStream_t st) {
  if (o.count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_assemble, dim3(blocks_for(o.count, 256)), dim3(256), 0, st, o.slot, o.entry, o.sid, o.count,
                     hv, sv, alpha, astride, o.npoles, hcoef, o.c, o.sc);
  return hipGetLastError();
}

// The op's descriptors come sorted by size class: count16 blocks with n <= 16,
// then count32 with n <= 32, then the rest (n <= 64).
hipError_t launch_smallinv(const DevOp& o, int* status, int spd_check, hipStream_t st) {
  const int64_t n16 = o.count16, n32 = o.count32, n64 = o.count - n16 - n32;
  if (n16 > 0)
    hipLaunchKernelGGL((k_smallinv<16, 64>), dim3(static_cast<unsigned>(n16), o.npoles), dim3(64), 0, st, o.inv, o.c,
                       o.sc, status, spd_check);
  if (n32 > 0)
    hipLaunchKernelGGL((k_smallinv<32, 128>), dim3(static_cast<unsigned>(n32), o.npoles), dim3(128), 0, st,
                       o.inv + n16, o.c, o.sc, status, spd_check);
  if (n64 > 0)
    hipLaunchKernelGGL((k_smallinv<64, 512>), dim3(static_cast<unsigned>(n64), o.npoles), dim3(512), 0, st,
                       o.inv + n16 + n32, o.c, o.sc, status, spd_check);
  return hipGetLastError();
}

template <int F>
static void gemm_inst(const DevOp& o, hipStream_t st) {
  const int64_t total = o.tile_count * o.npoles;
  if (o.small)  // two waves per 32x32 tile, two tiles per workgroup
    hipLaunchKernelGGL(k_zgemm_w<F>, dim3(static_cast<unsigned>((2 * total + 3) / 4)), dim3(256), 0, st, o.gemm,
                       o.gemm_tiles, o.tile_count, static_cast<int64_t>(o.npoles), o.a, o.sa, o.b, o.sb, o.c0, o.sc0,
                       o.c, o.sc, o.ext, o.ext_child, o.ext_inv);
  else
    hipLaunchKernelGGL(k_zgemm<F>, dim3(static_cast<unsigned>(total)), dim3(512), 0, st, o.gemm, o.gemm_tiles,
                       o.tile_count, static_cast<int64_t>(o.npoles), o.a, o.sa, o.b, o.sb, o.c0, o.sc0, o.c, o.sc, o.ext, o.ext_child, o.ext_inv);
}

template <int F>
static void gemm32_inst(const DevOp& o, hipStream_t st) {
  const int64_t total = o.tile_count * o.npoles;
  if (o.tile128)  // 128 x 128 tiles on sixteen waves of 32 x 32
    hipLaunchKernelGGL((k_cgemm32<F, 2, 4>), dim3(static_cast<unsigned>(total)), dim3(1024), 0, st, o.gemm, o.gemm_tiles,
                       o.tile_count, static_cast<int64_t>(o.npoles), o.a, o.sa, o.b, o.sb, o.c0, o.sc0, o.c, o.sc, o.ext, o.ext_child, o.ext_inv);
  else
    hipLaunchKernelGGL((k_cgemm32<F, 2, 2>), dim3(static_cast<unsigned>(total)), dim3(256), 0, st, o.gemm, o.gemm_tiles,
                       o.tile_count, static_cast<int64_t>(o.npoles), o.a, o.sa, o.b, o.sb, o.c0, o.sc0, o.c, o.sc, o.ext, o.ext_child, o.ext_inv);
}

template <int F>
static void gemm_bf3_inst(const DevOp& o, hipStream_t st) {
  const int64_t total = o.tile_count * o.npoles;
  if (o.bf3 == 1)
    hipLaunchKernelGGL((k_cgemm_bf3<F, 128, 8>), dim3(static_cast<unsigned>(total)), dim3(512), 0, st, o.gemm,
                       o.gemm_tiles, o.tile_count, static_cast<int64_t>(o.npoles), o.a, o.sa, o.b, o.sb, o.c0, o.sc0,
                       o.c, o.sc, o.ext, o.ext_child, o.ext_inv);
  else if (o.bf3 == 2)
    hipLaunchKernelGGL((k_cgemm_bf3<F, 64, 4>), dim3(static_cast<unsigned>(total)), dim3(256), 0, st, o.gemm,
                       o.gemm_tiles, o.tile_count, static_cast<int64_t>(o.npoles), o.a, o.sa, o.b, o.sb, o.c0, o.sc0,
                       o.c, o.sc, o.ext, o.ext_child, o.ext_inv);
  else if (o.bf3 == 3)
    hipLaunchKernelGGL(k_cgemm_bf3s<F>, dim3(static_cast<unsigned>(total)), dim3(512), 0, st, o.gemm, o.gemm_tiles,
                       o.tile_count, static_cast<int64_t>(o.npoles), o.a, o.sa, o.b, o.sb, o.c0, o.sc0, o.c, o.sc, o.ext, o.ext_child, o.ext_inv);
  else if (o.bf3 == 5)
    hipLaunchKernelGGL(k_cgemm_bf3w<F>, dim3(static_cast<unsigned>(total)), dim3(1024), 0, st, o.gemm, o.gemm_tiles,
                       o.tile_count, static_cast<int64_t>(o.npoles), o.a, o.sa, o.b, o.sb, o.c0, o.sc0, o.c, o.sc, o.ext, o.ext_child, o.ext_inv);
  else
    hipLaunchKernelGGL(k_cgemm_bf3p<F>, dim3(static_cast<unsigned>(total)), dim3(512), 0, st, o.gemm, o.gemm_tiles,
                       o.tile_count, static_cast<int64_t>(o.npoles), o.a, o.sa, o.b, o.sb, o.c0, o.sc0, o.c, o.sc, o.ext, o.ext_child, o.ext_inv);
}

hipError_t launch_gemm(const DevOp& o, hipStream_t st) {
  if (o.tile_count == 0) return hipSuccess;
  if (o.a32 && (o.flags != (G_NEG | G_SYMA) || !(o.bf3 || o.fp32))) return hipErrorInvalidValue;
  if (o.bf3) {
    switch (o.flags) {  // front updates and pivot-inverse products
      case 0: gemm_bf3_inst<0>(o, st); break;
      case G_NEG: gemm_bf3_inst<G_NEG>(o, st); break;
      case G_TB | G_SYM | G_BETA | G_NEG: gemm_bf3_inst<G_TB | G_SYM | G_BETA | G_NEG>(o, st); break;
      case G_NEG | G_SYMA:
        if (o.a32) gemm_bf3_inst<G_NEG | G_SYMA | G_A32>(o, st);
        else gemm_bf3_inst<G_NEG | G_SYMA>(o, st);
        break;
      case G_TB | G_SYM | G_EXTC0 | G_NEG | G_NOMIRROR: gemm_bf3_inst<G_TB | G_SYM | G_EXTC0 | G_NEG | G_NOMIRROR>(o, st); break;
      case G_TA | G_SYM | G_BETA | G_NEG: gemm_bf3_inst<G_TA | G_SYM | G_BETA | G_NEG>(o, st); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (o.fp32) {
    switch (o.flags) {  // front updates and pivot-inverse products
      case 0: gemm32_inst<0>(o, st); break;
      case G_NEG: gemm32_inst<G_NEG>(o, st); break;
      case G_TB | G_SYM | G_BETA | G_NEG: gemm32_inst<G_TB | G_SYM | G_BETA | G_NEG>(o, st); break;
      case G_NEG | G_SYMA:
        if (o.a32) gemm32_inst<G_NEG | G_SYMA | G_A32>(o, st);
        else gemm32_inst<G_NEG | G_SYMA>(o, st);
        break;
      case G_TB | G_SYM | G_EXTC0 | G_NEG | G_NOMIRROR: gemm32_inst<G_TB | G_SYM | G_EXTC0 | G_NEG | G_NOMIRROR>(o, st); break;
      case G_TA | G_SYM | G_BETA | G_NEG: gemm32_inst<G_TA | G_SYM | G_BETA | G_NEG>(o, st); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (o.flags) {
    case 0: gemm_inst<0>(o, st); break;
    case G_NEG: gemm_inst<G_NEG>(o, st); break;
    case G_NEG | G_SYMA: gemm_inst<G_NEG | G_SYMA>(o, st); break;
    case G_TB | G_SYM | G_EXTC0 | G_NEG | G_NOMIRROR: gemm_inst<G_TB | G_SYM | G_EXTC0 | G_NEG | G_NOMIRROR>(o, st); break;
    case G_TB | G_SYM | G_BETA | G_NEG: gemm_inst<G_TB | G_SYM | G_BETA | G_NEG>(o, st); break;
    case G_TA | G_SYM | G_BETA | G_NEG: gemm_inst<G_TA | G_SYM | G_BETA | G_NEG>(o, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_copy(const DevOp& o, hipStream_t st) {
  if (o.tile_count == 0) return hipSuccess;
  if (o.flags & 1)
    hipLaunchKernelGGL(k_copy<true>, dim3(static_cast<unsigned>(o.tile_count), o.npoles), dim3(256), 0, st, o.copy,
                       o.copy_tiles, o.a, o.sa, o.c, o.sc);
  else
    hipLaunchKernelGGL(k_copy<false>, dim3(static_cast<unsigned>(o.tile_count), o.npoles), dim3(256), 0, st, o.copy,
                       o.copy_tiles, o.a, o.sa, o.c, o.sc);
  return hipGetLastError();
}

hipError_t launch_gather(const DevOp& o, hipStream_t st) {
  if (o.tile_count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3(static_cast<unsigned>(o.tile_count), o.npoles), dim3(256), 0, st, o.gat, o.rel,
                     o.elem_tiles, o.a, o.sa, o.b, o.sb, o.c, o.sc, o.nhi, o.gat_in32, o.gat_out32);
  return hipGetLastError();
}

hipError_t launch_accum(const int64_t* slot, int64_t count, const double2* panel, int64_t ps, const double* w,
                        int npoles, double* acc, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_accum, dim3(blocks_for(count, 256)), dim3(256), 0, st, slot, count, panel, ps, w, npoles, acc);
  return hipGetLastError();
}

hipError_t launch_init_acc(const double* m0, int64_t count, int add_m0, double* acc, int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_init_acc, dim3(blocks_for(count > 4 ? count : 4, 256)), dim3(256), 0, st, m0, count, add_m0, acc,
                     status);
  return hipGetLastError();
}

hipError_t launch_scatter(const int32_t* entry, int64_t count, const double* acc, double* out, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3(blocks_for(count, 256)), dim3(256), 0, st, entry, count, acc, out);
  return hipGetLastError();
}

}  // namespace ndrho
