// Device-side views of the plan descriptors and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"

namespace ndrho {

// One resolved launch: descriptor pointers already offset to the op's range,
// buffers already resolved to (base pointer, pole stride).
struct DevOp {
  int flags = 0;
  int npoles = 1;
  bool a32 = false;      // GEMM: A operand stored as FP32 complex (G_A32)
  int64_t nhi = 0;       // GATHER: the first nhi poles keep FP64 G_UU
  int gat_in32 = 0;      // GATHER: the parent's G_UU of the other poles is FP32
  int gat_out32 = 0;     // GATHER: write the G_UU of the other poles as FP32
  bool fp32 = false;     // GEMM products on the FP32 matrix cores
  bool tile128 = false;  // FP32 GEMM on 128x128 tiles (else 64x64)
  bool small = false;    // FP64 GEMM with two waves per 32x32 tile, no LDS
  int bf3 = 0;           // split-BF16 products: 0 no; 1 128x128 tiles on 8 waves; 2 64x64 tiles on 4;
                         // 3 128x128 tiles, one split per element and stage; 4 128x128 tiles, K by
                         // 16 in double-buffered bf16 planes (needs Op::off32); 5 the same on sixteen
                         // waves of 32 x 32
  int64_t count = 0, tile_count = 0;
  int64_t count16 = 0, count32 = 0;  // pivot inverse: blocks of the n <= 16 and n <= 32 classes
  const GemmProb* gemm = nullptr;
  const TileRef* gemm_tiles = nullptr;
  const InvDesc* inv = nullptr;
  const CopyDesc* copy = nullptr;
  const CopyTile* copy_tiles = nullptr;
  const ExtAddDesc* ext = nullptr;
  const ExtAddChild* ext_child = nullptr;
  const int32_t* ext_inv = nullptr;
  const ElemTile* elem_tiles = nullptr;
  const GatherDesc* gat = nullptr;
  const int32_t* rel = nullptr;
  const int64_t* slot = nullptr;
  const int32_t* entry = nullptr;
  const int32_t* sid = nullptr;
  double2 *a = nullptr, *b = nullptr, *c0 = nullptr, *c = nullptr;
  int64_t sa = 0, sb = 0, sc0 = 0, sc = 0;
};

// ---- selected eigenstates (eigen.hip): block vectors of EIG_NR columns
constexpr int EIG_NR = 16;     // columns of a block vector
constexpr int EIG_GROWS = 16;  // rows of a forward-gather tile (EIG_GROWS x EIG_NR threads)
// One front of the solve through the stored factor, fronts ordered by depth.
struct SolveFront {
  int64_t j0;     // first pivot row (permuted position)
  int64_t w_off;  // its update rows' block in the update buffer (complex elements, EIG_NR per row)
  int32_t nj, nu, child_begin, child_count;
};
struct SolveChild {
  int64_t w_off;    // the child's update block (complex elements)
  int64_t inv_off;  // its inverse map over the parent's local rows (J then U): child update row or -1
  int32_t nu, pad;
};
struct SolveTile {  // EIG_GROWS local rows of one front
  int32_t front, r0;
};
// C rows (c_off + r) = [C0 rows (c0_off + r)] +/- op(A) B, A at a_off (column-major, lda), B rows b_off + k
// (or idx[b_off + k]); row offsets count rows of EIG_NR complex values.
struct TsProb {
  int64_t a_off, b_off, c_off, c0_off;
  int32_t lda, m, k, pad;
};
struct TsTile {  // 64 rows of one problem
  int32_t prob, m0;
};
enum { TS_FORWARD = 0, TS_DIAGONAL = 1, TS_BACKWARD = 2 };
hipError_t launch_spmm_perm(const int64_t* rp, const int32_t* col, const double* a, const int32_t* perm, int64_t n,
                            const double* x, double2* y, hipStream_t st);
hipError_t launch_spmm2(const int64_t* rp, const int32_t* col, const double* a, int64_t n, const double* x, double* w,
                        hipStream_t st);
hipError_t launch_solve_gather(const SolveFront* fronts, const SolveChild* kids, const int32_t* inv,
                               const SolveTile* tiles, int64_t ntiles, const double2* y, double2* z, double2* w,
                               hipStream_t st);
hipError_t launch_tsgemm(int mode, const TsProb* probs, const TsTile* tiles, int64_t ntiles, const double2* A,
                         const double2* B, const int32_t* idx, const double2* C0, double2* C, hipStream_t st);
hipError_t launch_unperm_split(const double2* x, const int32_t* iperm, int64_t n, double* v, hipStream_t st);
hipError_t launch_gram(const double* V, const double* W, int64_t n, int64_t chunk, int nblk, double* part,
                       hipStream_t st);
hipError_t launch_combine(const double* V, const double* Y, int64_t n, double* out, hipStream_t st);
hipError_t launch_resid(const double* hc, const double* sc, const double* theta, int64_t n, int64_t chunk, int nblk,
                        double* part, hipStream_t st);

// ---- fused kernels of the small fronts (smallfront.hip): one launch per depth
// and direction, one workgroup per (front, pole)
struct SmallLaunch {
  bool up = true;
  const SmallFront* fronts = nullptr;  // the fronts of one depth
  const SmallChild* kids = nullptr;
  const int32_t* inv = nullptr;
  const int32_t* rel = nullptr;
  int64_t nfronts = 0;
  int npoles = 0;
  double2 *panel = nullptr, *lbuf = nullptr, *upd0 = nullptr, *upd1 = nullptr;
  int64_t ps = 0, ls = 0, us = 0;
  const int64_t* asm_slot = nullptr;
  const int32_t* asm_entry = nullptr;
  const int32_t* asm_sid = nullptr;
  const double *hv = nullptr, *sv = nullptr;
  const double2* alpha = nullptr;
  int64_t astride = 0;
  double hcoef = 1.0;
  int spd_check = 0;
  int* status = nullptr;           // [0] singular pivots, [1] non-positive pivots of S
};
hipError_t launch_small(const SmallLaunch& s, hipStream_t st);

hipError_t launch_extadd(const DevOp& o, hipStream_t st);
hipError_t launch_assemble(const DevOp& o, const double* hv, const double* sv, const double2* alpha,
                           int64_t astride, double hcoef, hipStream_t st);
hipError_t launch_smallinv(const DevOp& o, int* status, int spd_check, hipStream_t st);
hipError_t launch_gemm(const DevOp& o, hipStream_t st);
hipError_t launch_copy(const DevOp& o, hipStream_t st);
hipError_t launch_gather(const DevOp& o, hipStream_t st);
hipError_t launch_accum(const int64_t* slot, int64_t count, const double2* panel, int64_t ps, const double* w,
                        int npoles, double* acc, hipStream_t st);
hipError_t launch_init_acc(const double* m0, int64_t count, int add_m0, double* acc, int* status, hipStream_t st);
hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, hipStream_t st);
hipError_t launch_scatter(const int32_t* entry, int64_t count, const double* acc, double* out, hipStream_t st);
// energy density matrix (energy.hip): acc_e = m1 + kappa m0, then acc_e += sum_p Re(cw_p G_p)
hipError_t launch_init_edm(const double* m1, const double* m0, double kappa, int64_t count, double* acc_e,
                           hipStream_t st);
// Tr(G_p S) per pole (trace.hip): partial[p * nblk + b], b < nblk, summed by the host
hipError_t launch_trace_gs(const int64_t* slot, const int32_t* entry, int64_t count, const double2* panel, int64_t ps,
                           const double* s, int npoles, int nblk, double2* partial, hipStream_t st);
hipError_t launch_accum_edm(const int64_t* slot, int64_t count, const double2* panel, int64_t ps,
                            const double2* cw, int npoles, const int32_t* ssid, int64_t cstride, double* acc_e,
                            hipStream_t st);

}  // namespace ndrho
