// Host-side plan: nested-dissection ordering, front tree, index maps and the
// launch program replayed by the device executor for every pole batch.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "common.h"

namespace ndrho {

void cf_poles(int n_poles, double* z, double* r);

// One front of the dissection tree (a domain at the innermost level or a
// separator, Sec. II C 1).  Its pivot rows J are the contiguous permuted
// positions [j0, j0 + nj); its update rows U (permuted positions, increasing)
// are the rows of ancestor separators coupled to its subtree.
struct Front {
  int parent = -1;
  int depth = 0;
  int64_t j0 = 0;
  int nj = 0;
  int nu = 0;
  std::vector<int> u;         // update rows (permuted positions)
  std::vector<int> rel;       // index of each u in the parent's (J, U) local order
  std::vector<int> children;
  int64_t panel_off = 0;      // column-major (nj+nu) x nj panel, per pole
  int64_t upd_off = 0;        // nu x nu update / gathered-G block in the depth's buffer
  int64_t temp_off = 0;       // scratch region in the temp buffer (recursive pivot inverse)
  int64_t l_off = 0;          // L_UJ = B A^{-1} (nu x nj, column-major, ld nu) in the L buffer
};

// Work descriptors shared with the device code (plain structs, 8-byte aligned).
struct GemmProb {
  int32_t m, n, k, lda, ldb, ldc0, ldc;
  int32_t ext;  // G_EXTC0: index of the front's extend-add descriptor (its children)
  int64_t a_off, b_off, c0_off, c_off;
};
struct TileRef {  // one 64x64 (or 128x128, or 32x32) output tile of problem `prob`
  int32_t prob, tm, tn, pad;
};
struct InvDesc {  // in-place inverse of an n x n block (n <= 64)
  int64_t off;
  int32_t ld, n;
};
struct CopyDesc {  // dst (rows x cols) <- src or src^T
  int64_t src_off, dst_off;
  int32_t lds, ldd, rows, cols;
};
struct CopyTile {
  int32_t desc, r0, c0, pad;
};
// Extend-add target: front p, whose children's update matrices are pulled
// into its panel (columns in J) and its own update block (U x U).
struct ExtAddDesc {
  int64_t panel_off, upd_off;
  int32_t nj, nu, child_begin, child_count;
};
struct ExtAddChild {
  int64_t upd_off;     // child's update block in the deeper buffer
  int64_t inv_off;     // into the inverse-map array: parent local index -> child U index or -1
  int32_t nu, pad;
};
struct ElemTile {     // 1024 consecutive target elements of descriptor `desc`
  int32_t desc;
  int32_t pad;
  int64_t e0;
};
// Gather of G_UU for front f from its parent p (downward pass).
struct GatherDesc {
  int64_t dst_off;          // f's block in the depth buffer
  int64_t rel_off;          // into the rel array
  int64_t ppanel_off;       // parent's panel
  int64_t pguu_off;         // parent's gathered G_UU in the shallower buffer
  int32_t nu, pnj, pnu, pad;
};

// One small front of a fused small-front launch (lists ordered by depth,
// deepest first for the upward launches, top first for the downward ones).
struct SmallFront {
  int64_t panel_off, l_off, upd_off;  // upd_off: its own update / G_UU block in its depth's buffer
  int64_t asm_begin, asm_end;         // its assembly entries (sorted tables)
  int64_t rel_off;                    // its relative map into the parent's local rows
  int64_t ppanel_off, pguu_off;       // the parent's panel and G_UU block
  int32_t nj, nu, depth;
  int32_t child_begin, child_count;   // its children (all small) in the child table
  int32_t parent_small;               // 1: the parent is small (the downward step gathers G_UU itself)
  int32_t pnj, pnu;
};
struct SmallChild {
  int64_t upd_off;  // the child's update block (in the child's depth buffer)
  int64_t inv_off;  // its inverse map over the parent's local rows (child update row or -1)
  int32_t nu, pad;
};

enum BufId { BUF_PANEL = 0, BUF_UPD0 = 1, BUF_UPD1 = 2, BUF_TEMP = 3, BUF_L = 4, BUF_COUNT = 5 };

enum OpKind { OP_EXTADD, OP_ASSEMBLE, OP_SMALLINV, OP_GEMM, OP_COPY, OP_GATHER, OP_SMALL };

// G_SYMA: A is symmetric and only its lower triangle is stored (entry (m, k)
// is read from (max, min)); G_NOMIRROR: with G_SYM, write the lower triangle
// of C only; G_EXTC0: C0 is not read but formed in the epilogue as the sum of
// the children's update entries that map onto (m, n) (the extend-add of the
// front's own U x U block, children in order).
enum GemmFlags { G_TA = 1, G_TB = 2, G_SYM = 4, G_BETA = 8, G_NEG = 16, G_NOMIRROR = 32, G_SYMA = 64,
                 G_EXTC0 = 128,
                 G_A32 = 512 };  // set at launch: the A operand is stored as FP32 complex (low-precision poles)
// Op-level marker (not a kernel flag): the GEMM belongs to a pivot-block
// inverse and always runs in FP64.
constexpr int OP_PIVOT = 1 << 8;

struct Op {
  OpKind kind;
  int flags = 0;             // GEMM variant, COPY transpose flag
  int buf_a = 0, buf_b = 0, buf_c0 = 0, buf_c = 0;  // for EXTADD: c = panel, a = child upd, b = own upd
  int64_t begin = 0, count = 0;          // descriptor range
  int64_t tile_begin = 0, tile_count = 0;
  int64_t tile128_begin = 0, tile128_count = 0;  // 128x128 tiles (FP32-product GEMMs)
  int64_t tile32_begin = 0, tile32_count = 0;    // 32x32 tiles (FP64 GEMM of small problems)
  bool small = false;        // GEMM: FP64 launches on 32x32 tiles by default (more than half of
                             // the 64x64 tile area would lie outside the problems)
  bool off32 = true;         // GEMM: every operand element of every problem lies within 2^31 - 16
                             // bytes of the problem's operand origin (32-bit offsets suffice)
  int64_t inv16 = 0, inv32 = 0;  // SMALLINV: leading descriptors with n <= 16, then n <= 32
  bool keep64 = false;       // GATHER: the G_UU it writes stays FP64 (its consumer is a small-front launch)
  int depth = 0;
  double flops = 0;          // useful flops per pole (GEMM, SMALL)
  double bytes = 0;          // algorithmic bytes per pole: operands read and results written once, complex128
};

struct Plan {
  int64_t n = 0, nnz = 0;
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> col;
  std::vector<int32_t> perm, iperm;
  std::vector<Front> fronts;   // postorder
  int n_levels = 0;
  int64_t panel_total = 0;     // complex elements per pole
  int64_t upd_total = 0;       // per depth buffer, complex elements per pole (max over depths)
  int64_t temp_total = 0;
  int64_t l_total = 0;         // complex elements per pole of the L buffer
  std::vector<int64_t> out_slot, asm_slot;   // per CSR entry

  // device program
  std::vector<Op> upward, downward;
  std::vector<GemmProb> gemm;
  std::vector<TileRef> gemm_tiles;
  std::vector<InvDesc> inv;
  std::vector<CopyDesc> copy;
  std::vector<CopyTile> copy_tiles;
  std::vector<ExtAddDesc> ext;
  std::vector<ExtAddChild> ext_child;
  std::vector<int32_t> ext_inv;
  std::vector<ElemTile> ext_tiles, gat_tiles;
  std::vector<GatherDesc> gat;
  std::vector<int32_t> rel_all;
  // assembly entries grouped by depth (sorted by slot within a depth)
  std::vector<int64_t> asm_slot_sorted;
  std::vector<int32_t> asm_entry_sorted;
  std::vector<int64_t> asm_depth_begin;       // n_levels + 1
  // accumulation entries sorted by slot
  std::vector<int64_t> acc_slot;
  std::vector<int32_t> acc_entry;

  double flops_model = 0, bytes_model = 0;    // per pole
  double flops_exec = 0;                      // flops of the program per pole

  // fused small-front launches (OP_SMALL, one per depth and direction: flags 0
  // upward, 1 downward; begin/count index small_up or small_down, which hold
  // the small fronts by depth, deepest first upward, top first downward)
  bool small_enabled = true;
  std::vector<SmallFront> small_up, small_down;
  std::vector<SmallChild> small_kids;
  std::vector<int32_t> small_inv;

  // several structures joined into one forest (empty for one structure):
  // first row / first CSR entry of each structure, and the structure of
  // every assembly entry (for per-structure shifts)
  std::vector<int64_t> struct_row_off, struct_nnz_off;
  std::vector<int32_t> asm_sid_sorted;
};

// Validate the CSR pattern (and values if given); throws Error(EINVAL).
void validate_csr(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* h, const double* s);
// Ordering + symbolic analysis + program.
// long_tail: rows whose pattern degree inside a domain exceeds long_tail
// times the domain's median join that domain's separator first (0: off).
// cell: NULL, or the periodic cell length along x, y, z (0: open boundary)
// for the coordinates in coords.
void build_plan(Plan& plan, int64_t n, const int64_t* row_ptr, const int32_t* col, const double* coords,
                int leaf_rows, double long_tail = 0.0, const double* cell = nullptr, bool small_fronts = false);
// Small fronts: at most 64 pivot rows and at most this many pivot plus update rows
constexpr int kSmallFrontRows = 320;
// Layout, tables and program from P's fronts and CSR (called by build_plan).
void finalize_plan(Plan& P);
// One plan for several structures: their front trees side by side as a
// forest over the block-diagonal union of their matrices.
void join_plans(Plan& U, const std::vector<const Plan*>& parts);

}  // namespace ndrho
