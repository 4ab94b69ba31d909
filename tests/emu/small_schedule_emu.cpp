// Host emulation of the fused small-front launches (csrc/smallfront.hip)
// through the stand-in HIP header: builds the plan of one structure whose
// fronts are all small, runs its upward and downward launches (one per depth
// and direction, in program order) over one shift alpha (X = alpha S -
// hcoef H) and writes G on the pattern in CSR order.
//
// Input file (native endianness): int64 n, nnz, has_cell; int64 row_ptr[n+1];
// int32 col[nnz]; double coords[3n]; double cell[3] if has_cell; double
// h[nnz], s[nnz]; double alpha_re, alpha_im, hcoef.
// Output file: double (re, im) per pattern entry, then int32 status[2].
// Exit code 2: the plan has fronts outside the fused small-front launches.
#include <cstdio>
#include <fstream>
#include <vector>

#include "hip/hip_runtime.h"
#include "kernels.h"
#include "plan.h"

using namespace ndrho;

int main(int argc, char** argv) {
  if (argc != 3) return 1;
  std::ifstream f(argv[1], std::ios::binary);
  int64_t n = 0, nnz = 0, has_cell = 0;
  f.read(reinterpret_cast<char*>(&n), 8);
  f.read(reinterpret_cast<char*>(&nnz), 8);
  f.read(reinterpret_cast<char*>(&has_cell), 8);
  std::vector<int64_t> rp(n + 1);
  std::vector<int32_t> col(nnz);
  std::vector<double> xyz(3 * n), cell(3, 0.0), h(nnz), s(nnz);
  f.read(reinterpret_cast<char*>(rp.data()), 8 * (n + 1));
  f.read(reinterpret_cast<char*>(col.data()), 4 * nnz);
  f.read(reinterpret_cast<char*>(xyz.data()), 24 * n);
  if (has_cell) f.read(reinterpret_cast<char*>(cell.data()), 24);
  f.read(reinterpret_cast<char*>(h.data()), 8 * nnz);
  f.read(reinterpret_cast<char*>(s.data()), 8 * nnz);
  double2 alpha;
  double hcoef = 1.0;
  f.read(reinterpret_cast<char*>(&alpha.x), 8);
  f.read(reinterpret_cast<char*>(&alpha.y), 8);
  f.read(reinterpret_cast<char*>(&hcoef), 8);
  if (!f) return 1;

  Plan P;
  build_plan(P, n, rp.data(), col.data(), xyz.data(), 32, 0.0, has_cell ? cell.data() : nullptr, true);
  for (const Op& op : P.upward)
    if (op.kind != OP_SMALL) return 2;
  for (const Op& op : P.downward)
    if (op.kind != OP_SMALL) return 2;
  std::vector<double2> panel(P.panel_total), lbuf(P.l_total), u0(P.upd_total), u1(P.upd_total);
  std::vector<int> status(4, 0);
  for (int pass = 0; pass < 2; ++pass)
    for (const Op& op : pass == 0 ? P.upward : P.downward) {
      SmallLaunch sl;
      sl.up = pass == 0;
      sl.fronts = (sl.up ? P.small_up.data() : P.small_down.data()) + op.begin;
      sl.kids = P.small_kids.data();
      sl.inv = P.small_inv.data();
      sl.rel = P.rel_all.data();
      sl.nfronts = op.count;
      sl.npoles = 1;
      sl.panel = panel.data(), sl.ps = P.panel_total;
      sl.lbuf = lbuf.data(), sl.ls = P.l_total;
      sl.upd0 = u0.data(), sl.upd1 = u1.data(), sl.us = P.upd_total;
      sl.asm_slot = P.asm_slot_sorted.data();
      sl.asm_entry = P.asm_entry_sorted.data();
      sl.asm_sid = P.asm_sid_sorted.data();
      sl.hv = h.data(), sl.sv = s.data();
      sl.alpha = &alpha, sl.astride = 0, sl.hcoef = hcoef, sl.spd_check = 0;
      sl.status = status.data();
      if (launch_small(sl, nullptr) != hipSuccess) return 1;
    }
  std::ofstream o(argv[2], std::ios::binary);
  for (int64_t e = 0; e < nnz; ++e) {
    const double2 v = panel[P.out_slot[e]];
    o.write(reinterpret_cast<const char*>(&v), sizeof(v));
  }
  o.write(reinterpret_cast<const char*>(status.data()), 2 * sizeof(int));
  return o ? 0 : 1;
}
