// Nested dissection (Sec. II C 1), symbolic front tree, the table from pattern
// entries to front positions (Sec. II C 2) and the launch program of the block
// LDL^T factorization and selected inversion (Eqs. (18)-(21), (38)-(39)).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <numeric>

#include "plan.h"

namespace ndrho {

// ----------------------------------------------------------------- validation

void validate_csr(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* h, const double* s) {
  if (n < 1 || n > (int64_t(1) << 31) - 2) fail(NDRHO_EINVAL, "n must be in [1, 2^31-2]");
  if (!row_ptr || !col) fail(NDRHO_EINVAL, "row_ptr and col_idx are required");
  if (row_ptr[0] != 0) fail(NDRHO_EINVAL, "row_ptr[0] must be 0");
  for (int64_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) fail(NDRHO_EINVAL, "row_ptr must be non-decreasing");
  for (int64_t i = 0; i < n; ++i) {
    bool diag = false;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int32_t j = col[e];
      if (j < 0 || j >= n) fail(NDRHO_EINVAL, "column index out of range in row " + std::to_string(i));
      if (e > row_ptr[i] && col[e - 1] >= j)
        fail(NDRHO_EINVAL, "column indices must be strictly increasing in row " + std::to_string(i));
      if (j == i) diag = true;
    }
    if (!diag) fail(NDRHO_EINVAL, "missing diagonal entry in row " + std::to_string(i));
  }
  double hmax = 0, smax = 0;
  const int64_t nnz = row_ptr[n];
  for (int64_t e = 0; e < nnz; ++e) {
    if (h) {
      if (!std::isfinite(h[e])) fail(NDRHO_EINVAL, "non-finite H value");
      hmax = std::max(hmax, std::fabs(h[e]));
    }
    if (s) {
      if (!std::isfinite(s[e])) fail(NDRHO_EINVAL, "non-finite S value");
      smax = std::max(smax, std::fabs(s[e]));
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int32_t j = col[e];
      const int32_t* b = col + row_ptr[j];
      const int32_t* en = col + row_ptr[j + 1];
      const int32_t* it = std::lower_bound(b, en, static_cast<int32_t>(i));
      if (it == en || *it != i) fail(NDRHO_EINVAL, "pattern is not structurally symmetric");
      const int64_t et = row_ptr[j] + (it - b);
      if (h && std::fabs(h[e] - h[et]) > 1e-12 * hmax) fail(NDRHO_EINVAL, "H is not symmetric");
      if (s && std::fabs(s[e] - s[et]) > 1e-12 * smax) fail(NDRHO_EINVAL, "S is not symmetric");
    }
  }
}

// ----------------------------------------------------------- nested dissection
//
// Procedures (i)-(v) of Sec. II C 1.  Each domain is ordered along each axis
// by the centre coordinate (ties broken by the other two coordinates, then by
// index); the position in that order is the ordering number.  The nucleus is
// the function with the fewest overlaps inside the domain; the subdomain grows
// from the end of the ordering nearest to the nucleus one function at a time,
// and at each step N0 (subdomain), Ns (functions between the subdomain and the
// extreme ordering numbers of the functions overlapping it) and
// N1 = Nd - N0 - Ns give the measure |N0 - N1| + Ns.  The axis and size with
// the smallest measure are taken, and both subdomains are dissected again
// until they hold at most leaf_rows functions.  Long-tail screening (step
// (ii)) is optional (see dissect).
//
// Periodic cells (step (i)): along an axis with a cell length L > 0, a
// neighbour reached across the cell boundary (coordinate difference beyond
// L/2, the minimum image) carries the ordering number of its periodic image,
// q - Nd or q + Nd for its number q in the domain, so the overlap range of a
// subdomain can reach below 0 or beyond Nd - 1: the separator then holds the
// functions after the subdomain and those wrapped round to the other end of
// the order (two planes for a periodic lattice), and the other subdomain is
// what lies between.  A cut is kept only if no overlap joins the two
// subdomains; otherwise the axis is searched again without images.

namespace {

struct NdNode {
  std::vector<int> members;   // original indices
  std::vector<int> children;  // node ids
};

class Dissector {
 public:
  Dissector(int64_t n, const int64_t* rp, const int32_t* col, const double* coords, const double* cell, int leaf,
            double tail)
      : n_(n), rp_(rp), col_(col), leaf_(leaf), tail_(tail), xyz_(3 * n, 0.0), stamp_(n, -1), lab_(n, 0), pos_(n, 0),
        naxes_(coords ? 3 : 1) {
    if (coords) std::copy(coords, coords + 3 * n, xyz_.begin());
    for (int a = 0; a < 3; ++a) cell_[a] = (coords && cell) ? cell[a] : 0.0;
  }

  std::vector<int> run() {
    std::vector<int> all(n_);
    std::iota(all.begin(), all.end(), 0);
    std::vector<int> lists[3];
    for (int a = 0; a < naxes_; ++a) {
      lists[a] = all;
      sort_axis(lists[a], a);
    }
    return dissect(lists);
  }

  std::vector<NdNode> nodes;

 private:
  int64_t n_;
  const int64_t* rp_;
  const int32_t* col_;
  int leaf_;
  double tail_;  // long-tail screening: degree above tail_ times the domain's median (0: off)
  std::vector<double> xyz_;
  std::vector<int> stamp_, lab_, pos_;
  int naxes_;
  double cell_[3] = {0.0, 0.0, 0.0};  // periodic cell length per axis (0: open)
  int next_stamp_ = 0;

  // Without coordinates: the breadth-first distance inside the domain from a
  // pseudo-peripheral row serves as the single ordering axis (recomputed for
  // every domain); disconnected pieces are laid out one after another.
  void bfs_coordinate(const std::vector<int>& dom, int st) {
    for (int v : dom) xyz_[3 * v] = -1.0;
    auto bfs = [&](int src, double base) {
      std::deque<int> q{src};
      xyz_[3 * src] = base;
      int last = src;
      while (!q.empty()) {
        int v = q.front();
        q.pop_front();
        last = v;
        for (int64_t e = rp_[v]; e < rp_[v + 1]; ++e) {
          int u = col_[e];
          if (stamp_[u] == st && xyz_[3 * u] < 0) {
            xyz_[3 * u] = xyz_[3 * v] + 1.0;
            q.push_back(u);
          }
        }
      }
      return last;
    };
    double base = 0.0;
    for (int v : dom) {
      if (xyz_[3 * v] >= 0) continue;
      // two sweeps to find a far end of this piece, then the final distances
      std::vector<int> piece;
      int far = bfs(v, base);
      for (int u : dom)
        if (xyz_[3 * u] >= base) piece.push_back(u);
      for (int u : piece) xyz_[3 * u] = -1.0;
      far = bfs(far, base);
      double top = base;
      for (int u : piece) top = std::max(top, xyz_[3 * u]);
      base = top + 2.0;
    }
  }

  void sort_axis(std::vector<int>& v, int a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const double* x = xyz_.data();
    std::sort(v.begin(), v.end(), [x, a, b, c](int p, int q) {
      if (x[3 * p + a] != x[3 * q + a]) return x[3 * p + a] < x[3 * q + a];
      if (x[3 * p + b] != x[3 * q + b]) return x[3 * p + b] < x[3 * q + b];
      if (x[3 * p + c] != x[3 * q + c]) return x[3 * p + c] < x[3 * q + c];
      return p < q;
    });
  }

  int make_node(std::vector<int> members, std::vector<int> children) {
    std::sort(members.begin(), members.end());
    nodes.push_back(NdNode{std::move(members), std::move(children)});
    return static_cast<int>(nodes.size()) - 1;
  }

  std::vector<int> dissect(std::vector<int> (&lists)[3]) {
    const int nd = static_cast<int>(lists[0].size());
    if (nd == 0) return {};
    if (nd <= leaf_) return {make_node(lists[0], {})};
    const int st = next_stamp_++;
    for (int v : lists[0]) stamp_[v] = st;
    // (ii) screening: rows that overlap far more rows of the domain than is
    // typical (basis functions with a long tail) join the separator before
    // the dissection, so that they do not hide the sparse structure of the
    // others; the cut is then sought among the remaining rows
    std::vector<int> screened;
    if (tail_ > 0.0) {
      std::vector<int> deg(nd);
      for (int q = 0; q < nd; ++q) {
        const int v = lists[0][q];
        int d = 0;
        for (int64_t e = rp_[v]; e < rp_[v + 1]; ++e)
          if (col_[e] != v && stamp_[col_[e]] == st) ++d;
        deg[q] = d;
      }
      std::vector<int> sorted = deg;
      std::nth_element(sorted.begin(), sorted.begin() + nd / 2, sorted.end());
      const double limit = tail_ * std::max(1, sorted[nd / 2]);
      const int rest_st = next_stamp_++;
      int kept = 0;
      for (int q = 0; q < nd; ++q) kept += deg[q] > limit ? 0 : 1;
      if (kept > 0 && kept < nd) {
        for (int q = 0; q < nd; ++q) {
          const int v = lists[0][q];
          if (deg[q] > limit) screened.push_back(v);
          else stamp_[v] = rest_st;
        }
        for (int a = 0; a < naxes_; ++a) {
          std::vector<int> keep;
          keep.reserve(kept);
          for (int v : lists[a])
            if (stamp_[v] == rest_st) keep.push_back(v);
          lists[a].swap(keep);
        }
        std::vector<int> r = dissect_rest(lists, rest_st);
        return {make_node(std::move(screened), std::move(r))};
      }
    }
    return dissect_rest(lists, st);
  }

  // Ordering number of the neighbour u of v along axis a: its position, or
  // that of its periodic image when the overlap crosses the cell boundary.
  int image_pos(int v, int u, int a, int nd, bool images) const {
    const int q = pos_[u];
    if (!images || cell_[a] <= 0.0) return q;
    const double d = xyz_[3 * u + a] - xyz_[3 * v + a];
    if (d > 0.5 * cell_[a]) return q - nd;
    if (d < -0.5 * cell_[a]) return q + nd;
    return q;
  }

  // Steps (iv)-(v): the best cut over all axes, as labels (0 subdomain,
  // 1 separator, 2 other subdomain) in lab_.  False when no axis has a cut
  // with a non-empty other subdomain.
  bool grow(std::vector<int> (&lists)[3], int st, int nucleus, bool images) {
    const int nd = static_cast<int>(lists[0].size());
    int64_t best_cost = -1, best_ns = 0;
    int best_axis = -1, best_cut = 0, best_end = 0, best_hi = 0, best_lo = 0;
    std::vector<int> hi(nd), lo(nd);
    for (int a = 0; a < naxes_; ++a) {
      const std::vector<int>& ord = lists[a];
      for (int q = 0; q < nd; ++q) pos_[ord[q]] = q;
      const bool low = pos_[nucleus] < nd - pos_[nucleus];
      for (int q = 0; q < nd; ++q) {
        const int v = ord[q];
        int h = q, l = q;
        for (int64_t e = rp_[v]; e < rp_[v + 1]; ++e) {
          const int u = col_[e];
          if (stamp_[u] != st) continue;
          const int p = image_pos(v, u, a, nd, images);
          h = std::max(h, p);
          l = std::min(l, p);
        }
        hi[q] = h;
        lo[q] = l;
      }
      auto consider = [&](int64_t n0, int64_t ns, int64_t n1, int m, int end, int nhi, int nlo) {
        const int64_t cost = std::llabs(n0 - n1) + ns;
        if (best_cost < 0 || cost < best_cost || (cost == best_cost && ns <= best_ns && a == best_axis)) {
          best_cost = cost, best_ns = ns, best_axis = a, best_cut = m, best_end = end, best_hi = nhi, best_lo = nlo;
        }
      };
      if (low) {
        int nmax = -1, nmin = 0;
        for (int m = 1; m < nd; ++m) {  // subdomain = ordering numbers [0, m)
          nmax = std::max(nmax, hi[m - 1]);
          nmin = std::min(nmin, lo[m - 1]);
          // separator: (m - 1, nmax] and, wrapped, [nd + nmin, nd)
          const int64_t n0 = m, ns = int64_t(nmax) - nmin + 1 - m, n1 = nd - n0 - ns;
          if (n1 < 1) break;
          consider(n0, ns, n1, m, 0, nmax, nmin);
        }
      } else {
        int nmin = nd, nmax = nd - 1;
        for (int m = nd - 1; m >= 1; --m) {  // subdomain = ordering numbers [m, nd)
          nmin = std::min(nmin, lo[m]);
          nmax = std::max(nmax, hi[m]);
          // separator: [nmin, m) and, wrapped, [0, nmax - nd]
          const int64_t n0 = nd - m, ns = int64_t(nmax) - nmin + 1 - n0, n1 = nd - n0 - ns;
          if (n1 < 1) break;
          consider(n0, ns, n1, m, 1, nmax, nmin);
        }
      }
    }
    if (best_axis < 0) return false;
    const std::vector<int>& ord = lists[best_axis];
    for (int q = 0; q < nd; ++q) {
      int l;
      if (best_end == 0) l = q < best_cut ? 0 : (q <= best_hi || q >= nd + best_lo) ? 1 : 2;
      else l = q >= best_cut ? 0 : (q >= best_lo || q <= best_hi - nd) ? 1 : 2;
      lab_[ord[q]] = l;
    }
    return true;
  }

  // No overlap between the two subdomains of the labels in lab_.
  bool separates(const std::vector<int> (&lists)[3], int st) const {
    for (int v : lists[0]) {
      if (lab_[v] == 1) continue;
      for (int64_t e = rp_[v]; e < rp_[v + 1]; ++e) {
        const int u = col_[e];
        if (stamp_[u] == st && lab_[u] != 1 && lab_[u] != lab_[v]) return false;
      }
    }
    return true;
  }

  // Steps (iii)-(v) on a domain whose rows carry the stamp `st`.
  std::vector<int> dissect_rest(std::vector<int> (&lists)[3], int st) {
    const int nd = static_cast<int>(lists[0].size());
    if (nd <= leaf_) return {make_node(lists[0], {})};
    if (naxes_ == 1) {
      bfs_coordinate(lists[0], st);
      sort_axis(lists[0], 0);
    }
    // (iii) nucleus: fewest overlaps with the other functions of the domain
    int nucleus = -1, best_deg = 1 << 30;
    for (int v : lists[0]) {
      int deg = 0;
      for (int64_t e = rp_[v]; e < rp_[v + 1]; ++e)
        if (col_[e] != v && stamp_[col_[e]] == st) ++deg;
      if (deg < best_deg || (deg == best_deg && v < nucleus)) {
        best_deg = deg;
        nucleus = v;
      }
    }
    // (iv)-(v) growth along each axis, with images across periodic cell
    // boundaries; the cut separates by construction, which is checked (and
    // the axes searched again without images should it not)
    const bool periodic = cell_[0] > 0.0 || cell_[1] > 0.0 || cell_[2] > 0.0;
    bool found = grow(lists, st, nucleus, periodic);
    if (found && periodic && !separates(lists, st)) found = grow(lists, st, nucleus, false);
    if (!found) return {make_node(lists[0], {})};  // no separating cut exists
    if (!separates(lists, st)) fail(NDRHO_EINVAL, "dissection produced a separator that does not separate");
    std::vector<int> sub[3][3];  // [label][axis]
    for (int a = 0; a < naxes_; ++a)
      for (int v : lists[a]) sub[lab_[v]][a].push_back(v);
    std::vector<int> sep = sub[1][0];
    for (int a = 0; a < 3; ++a) std::vector<int>().swap(lists[a]);
    std::vector<int> r0 = dissect(sub[0]);
    std::vector<int> r1 = dissect(sub[2]);
    r0.insert(r0.end(), r1.begin(), r1.end());
    if (sep.empty()) return r0;  // disconnected pieces: no separator front
    return {make_node(std::move(sep), std::move(r0))};
  }
};

int64_t rec_temp(int n) {
  if (n <= 64) return 0;
  const int nb = (n + 63) / 64;
  const int n1 = 64 * ((nb + 1) / 2), n2 = n - n1;
  return std::max(rec_temp(n1), static_cast<int64_t>(n2) * n1 + rec_temp(n2));
}

}  // namespace

// ----------------------------------------------------------------- program

namespace {

struct Builder {
  Plan& P;
  explicit Builder(Plan& p) : P(p) {}

  // one GEMM op over a list of problems
  void gemm(std::vector<Op>& prog, int flags, int ba, int bb, int bc0, int bc, const std::vector<GemmProb>& probs,
            int depth) {
    if (probs.empty()) return;
    Op op;
    op.kind = OP_GEMM;
    op.flags = flags;
    op.buf_a = ba, op.buf_b = bb, op.buf_c0 = bc0, op.buf_c = bc;
    op.begin = static_cast<int64_t>(P.gemm.size());
    op.count = static_cast<int64_t>(probs.size());
    op.tile_begin = static_cast<int64_t>(P.gemm_tiles.size());
    op.depth = depth;
    double fl = 0, by = 0;
    for (size_t i = 0; i < probs.size(); ++i) {
      const GemmProb& g = probs[i];
      P.gemm.push_back(g);
      // algorithmic bytes: A (lower triangle if stored so), B, C written (lower
      // triangle unless mirrored), C0 read with G_BETA, the children's
      // entries of a G_EXTC0 sum taken as one read per result element
      const double ea = (flags & G_SYMA) ? double(g.k) * (g.k + 1) / 2 : double(g.m) * g.k;
      const double ec = (flags & G_SYM) ? ((flags & G_NOMIRROR) ? double(g.n) * (g.n + 1) / 2 : double(g.m) * g.n)
                                        : double(g.m) * g.n;
      const double ec0 = (flags & G_SYM) ? double(g.n) * (g.n + 1) / 2 : double(g.m) * g.n;
      by += 16.0 * (ea + double(g.k) * g.n + ec + ((flags & (G_BETA | G_EXTC0)) ? ec0 : 0.0));
      const int tm = (g.m + 63) / 64, tn = (g.n + 63) / 64;
      for (int a = 0; a < tm; ++a)
        for (int b = 0; b < tn; ++b) {
          if ((flags & G_SYM) && b > a) continue;  // lower tiles only
          P.gemm_tiles.push_back(TileRef{static_cast<int32_t>(i), a, b, 0});
        }
      if (flags & G_SYM) fl += 8.0 * g.k * (double(g.n) * (g.n + 1) / 2);
      else fl += 8.0 * double(g.m) * g.n * g.k;
    }
    op.tile_count = static_cast<int64_t>(P.gemm_tiles.size()) - op.tile_begin;
    op.tile128_begin = static_cast<int64_t>(P.gemm_tiles.size());
    for (size_t i = 0; i < probs.size(); ++i) {  // for low-precision GEMMs on 128x128 tiles
      const GemmProb& g = probs[i];
      const int tm = (g.m + 127) / 128, tn = (g.n + 127) / 128;
      for (int a = 0; a < tm; ++a)
        for (int b = 0; b < tn; ++b) {
          if ((flags & G_SYM) && b > a) continue;
          P.gemm_tiles.push_back(TileRef{static_cast<int32_t>(i), a, b, 0});
        }
    }
    op.tile128_count = static_cast<int64_t>(P.gemm_tiles.size()) - op.tile128_begin;
    op.tile32_begin = static_cast<int64_t>(P.gemm_tiles.size());
    double area = 0;
    for (size_t i = 0; i < probs.size(); ++i) {
      const GemmProb& g = probs[i];
      const int tm = (g.m + 31) / 32, tn = (g.n + 31) / 32;
      for (int a = 0; a < tm; ++a)
        for (int b = 0; b < tn; ++b) {
          if ((flags & G_SYM) && b > a) continue;
          P.gemm_tiles.push_back(TileRef{static_cast<int32_t>(i), a, b, 0});
        }
      area += (flags & G_SYM) ? double(g.n) * (g.n + 1) / 2 : double(g.m) * g.n;
    }
    op.tile32_count = static_cast<int64_t>(P.gemm_tiles.size()) - op.tile32_begin;
    op.small = double(op.tile_count) * 64 * 64 > 2.0 * area;
    for (const GemmProb& g : probs) {  // largest byte offset of an operand element, either storage order
      const double ea = 16.0 * double(std::max(g.m, g.k)) * (double(g.lda) + 1.0);
      const double eb = 16.0 * double(std::max(g.n, g.k)) * (double(g.ldb) + 1.0);
      if (std::max(ea, eb) >= 2147483632.0) op.off32 = false;
    }
    op.flops = fl;
    op.bytes = by;
    P.flops_exec += fl;
    prog.push_back(op);
  }

  void copy(std::vector<Op>& prog, bool transpose, int bs, int bd, const std::vector<CopyDesc>& descs, int depth) {
    if (descs.empty()) return;
    Op op;
    op.kind = OP_COPY;
    op.flags = transpose ? 1 : 0;
    op.buf_a = bs, op.buf_c = bd;
    op.begin = static_cast<int64_t>(P.copy.size());
    op.count = static_cast<int64_t>(descs.size());
    op.tile_begin = static_cast<int64_t>(P.copy_tiles.size());
    op.depth = depth;
    for (size_t i = 0; i < descs.size(); ++i) {
      P.copy.push_back(descs[i]);
      for (int r = 0; r < descs[i].rows; r += 64)
        for (int c = 0; c < descs[i].cols; c += 64)
          P.copy_tiles.push_back(CopyTile{static_cast<int32_t>(i), r, c, 0});
    }
    op.tile_count = static_cast<int64_t>(P.copy_tiles.size()) - op.tile_begin;
    prog.push_back(op);
  }

  void smallinv(std::vector<Op>& prog, const std::vector<InvDesc>& descs, int depth) {
    if (descs.empty()) return;
    Op op;
    op.kind = OP_SMALLINV;
    op.buf_c = BUF_PANEL;
    op.begin = static_cast<int64_t>(P.inv.size());
    op.count = static_cast<int64_t>(descs.size());
    op.depth = depth;
    // sorted by size class (n <= 16, n <= 32, n <= 64), each on its own kernel
    for (int cls = 0; cls < 3; ++cls)
      for (const InvDesc& d : descs) {
        if (d.n < 1 || d.n > 64) throw Error(NDRHO_EINVAL, "pivot block size out of range");
        const int dc = d.n <= 16 ? 0 : d.n <= 32 ? 1 : 2;
        if (dc != cls) continue;
        P.inv.push_back(d);
        P.flops_exec += 8.0 * double(d.n) * d.n * d.n;
        if (cls == 0) ++op.inv16;
        if (cls == 1) ++op.inv32;
      }
    prog.push_back(op);
  }

  // In-place inverse of the leading n_f x n_f block (at row/column r0_f) of
  // each front f in `grp`, by the block form of Eq. (21) applied
  // recursively: A11^{-1}; L = A21 A11^{-1}; S = A22 - L A21^T; S^{-1};
  // G21 = -S^{-1} L; G11 = A11^{-1} - L^T G21; G12 = G21^T.  All blocks of a
  // group span the same number of 64-row blocks, so they share one split
  // (n1 = 64 ceil(blocks/2)) and every launch of the recursion serves the
  // whole group, each problem with its own sizes.
  void inverse(std::vector<Op>& prog, const std::vector<int>& grp, const std::vector<int>& n,
               const std::vector<int>& r0, const std::vector<int64_t>& tstack, int depth) {
    const int nb = (n[0] + 63) / 64;
    if (nb <= 1) {
      std::vector<InvDesc> d;
      for (size_t g = 0; g < grp.size(); ++g) {
        const Front& F = P.fronts[grp[g]];
        const int ld = F.nj + F.nu;
        d.push_back(InvDesc{F.panel_off + r0[g] + int64_t(r0[g]) * ld, ld, n[g]});
      }
      smallinv(prog, d, depth);
      return;
    }
    const int n1 = 64 * ((nb + 1) / 2);
    std::vector<int> n1v(grp.size(), n1), n2v(grp.size()), r1v(grp.size());
    std::vector<int64_t> t2v(grp.size());
    for (size_t g = 0; g < grp.size(); ++g) {
      n2v[g] = n[g] - n1;
      r1v[g] = r0[g] + n1;
      t2v[g] = tstack[g] + int64_t(n2v[g]) * n1;
    }
    inverse(prog, grp, n1v, r0, tstack, depth);
    auto at = [&](const Front& F, int r, int c) { return F.panel_off + r + int64_t(c) * (F.nj + F.nu); };
    std::vector<GemmProb> ga, gb, gc, gd;
    std::vector<CopyDesc> ct;
    for (size_t g = 0; g < grp.size(); ++g) {
      const Front& F = P.fronts[grp[g]];
      const int ld = F.nj + F.nu;
      const int n2 = n2v[g], a = r0[g];
      const int64_t t = F.temp_off + tstack[g];
      // L = A21 A11^{-1}   (n2 x n1)
      ga.push_back(GemmProb{n2, n1, n1, ld, ld, 0, n2, 0, at(F, a + n1, a), at(F, a, a), 0, t});
      // A22 <- A22 - L A21^T
      gb.push_back(GemmProb{n2, n2, n1, n2, ld, ld, ld, 0, t, at(F, a + n1, a), at(F, a + n1, a + n1),
                            at(F, a + n1, a + n1)});
      // A21 <- -S^{-1} L
      gc.push_back(GemmProb{n2, n1, n2, ld, n2, 0, ld, 0, at(F, a + n1, a + n1), t, 0, at(F, a + n1, a)});
      // A11 <- A11^{-1} - L^T G21
      gd.push_back(GemmProb{n1, n1, n2, n2, ld, ld, ld, 0, t, at(F, a + n1, a), at(F, a, a), at(F, a, a)});
      // A12 <- G21^T
      ct.push_back(CopyDesc{at(F, a + n1, a), at(F, a, a + n1), ld, ld, n1, n2});
    }
    gemm(prog, OP_PIVOT, BUF_PANEL, BUF_PANEL, 0, BUF_TEMP, ga, depth);
    gemm(prog, OP_PIVOT | G_TB | G_SYM | G_BETA | G_NEG, BUF_TEMP, BUF_PANEL, BUF_PANEL, BUF_PANEL, gb, depth);
    inverse(prog, grp, n2v, r1v, t2v, depth);
    gemm(prog, OP_PIVOT | G_NEG, BUF_PANEL, BUF_TEMP, 0, BUF_PANEL, gc, depth);
    gemm(prog, OP_PIVOT | G_TA | G_SYM | G_BETA | G_NEG, BUF_TEMP, BUF_PANEL, BUF_PANEL, BUF_PANEL, gd, depth);
    copy(prog, true, BUF_PANEL, BUF_PANEL, ct, depth);
  }
};

}  // namespace

void build_plan(Plan& P, int64_t n, const int64_t* row_ptr, const int32_t* col, const double* coords,
                int leaf_rows, double long_tail, const double* cell, bool small_fronts) {
  // (small_fronts: the small fronts run in the fused small-front launches)
  if (leaf_rows < 1) fail(NDRHO_EINVAL, "leaf_rows must be >= 1");
  if (!(long_tail == 0.0 || long_tail >= 1.0)) fail(NDRHO_EINVAL, "long_tail must be 0 or >= 1");
  P = Plan();
  P.small_enabled = small_fronts;
  P.n = n;
  P.nnz = row_ptr[n];
  P.row_ptr.assign(row_ptr, row_ptr + n + 1);
  P.col.assign(col, col + P.nnz);

  // ---- ordering
  if (cell)
    for (int a = 0; a < 3; ++a)
      if (!(cell[a] >= 0.0) || !std::isfinite(cell[a])) fail(NDRHO_EINVAL, "cell lengths must be finite and >= 0");
  Dissector nd(n, row_ptr, col, coords, cell, leaf_rows, long_tail);
  std::vector<int> roots = nd.run();
  std::vector<NdNode>& nodes = nd.nodes;
  // postorder: children (in order) before the node
  std::vector<int> post;
  post.reserve(nodes.size());
  {
    std::vector<std::pair<int, size_t>> stack;
    for (int r : roots) {
      stack.push_back({r, 0});
      while (!stack.empty()) {
        auto& top = stack.back();
        if (top.second < nodes[top.first].children.size()) {
          int c = nodes[top.first].children[top.second++];
          stack.push_back({c, 0});
        } else {
          post.push_back(top.first);
          stack.pop_back();
        }
      }
    }
  }
  std::vector<int> node2front(nodes.size(), -1);
  for (size_t i = 0; i < post.size(); ++i) node2front[post[i]] = static_cast<int>(i);
  P.fronts.resize(post.size());
  P.perm.resize(n);
  P.iperm.resize(n);
  int64_t next = 0;
  for (size_t i = 0; i < post.size(); ++i) {
    Front& F = P.fronts[i];
    const NdNode& nd_node = nodes[post[i]];
    F.j0 = next;
    F.nj = static_cast<int>(nd_node.members.size());
    for (int v : nd_node.members) {
      P.perm[next] = v;
      P.iperm[v] = static_cast<int32_t>(next);
      ++next;
    }
    for (int c : nd_node.children) {
      F.children.push_back(node2front[c]);
      P.fronts[node2front[c]].parent = static_cast<int>(i);
    }
  }
  if (next != n) fail(NDRHO_EINVAL, "dissection lost rows");
  const int nf = static_cast<int>(P.fronts.size());
  int maxdepth = 0;
  for (int f = nf - 1; f >= 0; --f) {
    Front& F = P.fronts[f];
    F.depth = F.parent < 0 ? 0 : P.fronts[F.parent].depth + 1;
    maxdepth = std::max(maxdepth, F.depth);
  }
  P.n_levels = maxdepth + 1;

  // ---- symbolic: update sets U_f and relative maps
  std::vector<int> owner(n, -1);
  for (int f = 0; f < nf; ++f)
    for (int64_t q = P.fronts[f].j0; q < P.fronts[f].j0 + P.fronts[f].nj; ++q) owner[q] = f;
  std::vector<int> mark(n, -1);
  for (int f = 0; f < nf; ++f) {
    Front& F = P.fronts[f];
    const int64_t end = F.j0 + F.nj;
    std::vector<int>& U = F.u;
    for (int64_t q = F.j0; q < end; ++q) {
      const int v = P.perm[q];
      for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        const int p = P.iperm[col[e]];
        if (p >= end && mark[p] != f) {
          mark[p] = f;
          U.push_back(p);
        }
      }
    }
    for (int c : F.children) {
      for (int p : P.fronts[c].u) {
        if (p < F.j0) fail(NDRHO_EINVAL, "dissection produced a separator that does not separate");
        if (p >= end && mark[p] != f) {
          mark[p] = f;
          U.push_back(p);
        }
      }
    }
    std::sort(U.begin(), U.end());
    F.nu = static_cast<int>(U.size());
    if (F.parent < 0 && F.nu != 0) fail(NDRHO_EINVAL, "root front with a non-empty update set");
    for (int c : F.children) {
      Front& C = P.fronts[c];
      C.rel.resize(C.nu);
      for (int k = 0; k < C.nu; ++k) {
        const int p = C.u[k];
        if (p < end) {
          C.rel[k] = static_cast<int>(p - F.j0);
        } else {
          auto it = std::lower_bound(U.begin(), U.end(), p);
          if (it == U.end() || *it != p) fail(NDRHO_EINVAL, "update set of a child is not closed in its parent");
          C.rel[k] = F.nj + static_cast<int>(it - U.begin());
        }
      }
    }
  }

  finalize_plan(P);
}

// Storage layout, the table of pattern positions and the launch program,
// from the front tree and the CSR pattern held in P (one structure, or the
// forest of several structures joined by join_plans).
void finalize_plan(Plan& P) {
  const int nf = static_cast<int>(P.fronts.size());
  std::vector<int> owner(P.n, -1);
  for (int f = 0; f < nf; ++f)
    for (int64_t q = P.fronts[f].j0; q < P.fronts[f].j0 + P.fronts[f].nj; ++q) owner[q] = f;
  P.flops_model = P.bytes_model = P.flops_exec = 0;
  P.upd_total = P.temp_total = 0;
  P.upward.clear();
  P.downward.clear();
  // ---- storage offsets
  std::vector<std::vector<int>> by_depth(P.n_levels);
  for (int f = 0; f < nf; ++f) by_depth[P.fronts[f].depth].push_back(f);
  int64_t po = 0;
  for (int f = 0; f < nf; ++f) {
    const Front& F = P.fronts[f];
    // the extend-add and gather kernels index a front's panel and update
    // block with 32-bit element numbers
    if (int64_t(F.nj + F.nu) * F.nj >= (int64_t(1) << 32) || int64_t(F.nu) * F.nu >= (int64_t(1) << 32))
      fail(NDRHO_EINVAL, "a front of " + std::to_string(F.nj) + " pivot and " + std::to_string(F.nu) +
                             " update rows exceeds 2^32 elements per block");
  }
  for (int f = 0; f < nf; ++f) {
    Front& F = P.fronts[f];
    F.panel_off = po;
    po += int64_t(F.nj + F.nu) * F.nj;
    P.flops_model += 8.0 * (double(F.nj) * F.nj * F.nj + double(F.nu) * F.nj * F.nj +
                            double(F.nu) * F.nu * F.nj / 2 + double(F.nu) * F.nu * F.nj +
                            double(F.nu) * F.nj * F.nj / 2);
    P.bytes_model += 16.0 * (2.0 * (double(F.nj) * F.nj + double(F.nu) * F.nj) + 3.0 * double(F.nu) * F.nu);
  }
  P.panel_total = po;
  int64_t lo = 0;
  for (int f = 0; f < nf; ++f) {
    Front& F = P.fronts[f];
    F.l_off = lo;
    lo += int64_t(F.nu) * F.nj;
  }
  P.l_total = std::max<int64_t>(lo, 1);
  // small fronts (those of the fused small-front launches): at most 64 pivot
  // rows, at most kSmallFrontRows pivot plus update rows, every descendant
  // small too
  // (postorder: children come first)
  std::vector<char> small(nf, 0);
  if (P.small_enabled)
    for (int f = 0; f < nf; ++f) {
      const Front& F = P.fronts[f];
      bool sm = F.nj <= 64 && F.nj + F.nu <= kSmallFrontRows;
      for (int c : F.children) sm = sm && small[c];
      small[f] = sm;
    }
  // update / G_UU blocks: the large fronts of a depth side by side in their
  // depth's buffer (reused by the depths of the same parity), every small
  // front a block of its own after them
  for (int d = 0; d < P.n_levels; ++d) {
    int64_t uo = 0, to = 0;
    for (int f : by_depth[d]) {
      Front& F = P.fronts[f];
      if (small[f]) continue;
      F.upd_off = uo;
      uo += int64_t(F.nu) * F.nu;
      F.temp_off = to;
      to += rec_temp(F.nj);
    }
    P.upd_total = std::max(P.upd_total, uo);
    P.temp_total = std::max(P.temp_total, to);
  }
  {
    int64_t so[2] = {P.upd_total, P.upd_total};
    for (int f = 0; f < nf; ++f) {
      Front& F = P.fronts[f];
      if (!small[f]) continue;
      F.upd_off = so[F.depth & 1];
      so[F.depth & 1] += int64_t(F.nu) * F.nu;
      F.temp_off = 0;
    }
    P.upd_total = std::max(P.upd_total, std::max(so[0], so[1]));
  }
  P.upd_total = std::max<int64_t>(P.upd_total, 1);
  P.temp_total = std::max<int64_t>(P.temp_total, 1);

  // ---- table of pattern positions (assembly and output slots)
  P.out_slot.resize(P.nnz);
  P.asm_slot.resize(P.nnz);
  std::vector<std::vector<std::pair<int64_t, int32_t>>> asm_by_depth(P.n_levels), asm_small(nf);
  for (int64_t i = 0; i < P.n; ++i) {
    for (int64_t e = P.row_ptr[i]; e < P.row_ptr[i + 1]; ++e) {
      const int pi = P.iperm[i], pj = P.iperm[P.col[e]];
      const int a = std::min(pi, pj), b = std::max(pi, pj);
      const Front& F = P.fronts[owner[a]];
      const int64_t ld = F.nj + F.nu;
      const int la = static_cast<int>(a - F.j0);
      if (b < F.j0 + F.nj) {
        const int li = static_cast<int>(pi - F.j0), lj = static_cast<int>(pj - F.j0);
        P.asm_slot[e] = F.panel_off + li + lj * ld;
        P.out_slot[e] = F.panel_off + std::max(li, lj) + std::min(li, lj) * ld;
      } else {
        auto it = std::lower_bound(F.u.begin(), F.u.end(), b);
        const int lb = F.nj + static_cast<int>(it - F.u.begin());
        const int64_t slot = F.panel_off + lb + la * ld;
        P.out_slot[e] = slot;
        P.asm_slot[e] = (pi == b) ? slot : -1;
      }
      if (P.asm_slot[e] >= 0) {
        if (small[owner[a]]) asm_small[owner[a]].push_back({P.asm_slot[e], static_cast<int32_t>(e)});
        else asm_by_depth[F.depth].push_back({P.asm_slot[e], static_cast<int32_t>(e)});
      }
    }
  }
  P.asm_depth_begin.assign(P.n_levels + 1, 0);
  for (int d = 0; d < P.n_levels; ++d) {
    auto& v = asm_by_depth[d];
    std::sort(v.begin(), v.end());
    P.asm_depth_begin[d] = static_cast<int64_t>(P.asm_slot_sorted.size());
    for (auto& pr : v) {
      P.asm_slot_sorted.push_back(pr.first);
      P.asm_entry_sorted.push_back(pr.second);
    }
  }
  P.asm_depth_begin[P.n_levels] = static_cast<int64_t>(P.asm_slot_sorted.size());
  // the small fronts' entries follow, front by front (sorted by slot)
  std::vector<int64_t> asm_small_begin(nf, 0), asm_small_end(nf, 0);
  for (int f = 0; f < nf; ++f) {
    if (!small[f]) continue;
    auto& v = asm_small[f];
    std::sort(v.begin(), v.end());
    asm_small_begin[f] = static_cast<int64_t>(P.asm_slot_sorted.size());
    for (auto& pr : v) {
      P.asm_slot_sorted.push_back(pr.first);
      P.asm_entry_sorted.push_back(pr.second);
    }
    asm_small_end[f] = static_cast<int64_t>(P.asm_slot_sorted.size());
  }
  P.asm_sid_sorted.assign(P.asm_entry_sorted.size(), 0);
  if (!P.struct_nnz_off.empty())
    for (size_t k = 0; k < P.asm_entry_sorted.size(); ++k)
      P.asm_sid_sorted[k] = static_cast<int32_t>(
          std::upper_bound(P.struct_nnz_off.begin(), P.struct_nnz_off.end(), int64_t(P.asm_entry_sorted[k])) -
          P.struct_nnz_off.begin() - 1);
  {
    std::vector<std::pair<int64_t, int32_t>> acc(P.nnz);
    for (int64_t e = 0; e < P.nnz; ++e) acc[e] = {P.out_slot[e], static_cast<int32_t>(e)};
    std::sort(acc.begin(), acc.end());
    P.acc_slot.resize(P.nnz);
    P.acc_entry.resize(P.nnz);
    for (int64_t k = 0; k < P.nnz; ++k) {
      P.acc_slot[k] = acc[k].first;
      P.acc_entry[k] = acc[k].second;
    }
  }

  // ---- relative maps, concatenated
  std::vector<int64_t> rel_off(nf, 0);
  for (int f = 0; f < nf; ++f) {
    rel_off[f] = static_cast<int64_t>(P.rel_all.size());
    P.rel_all.insert(P.rel_all.end(), P.fronts[f].rel.begin(), P.fronts[f].rel.end());
  }

  // ---- fused small-front launches: the small fronts by depth, deepest
  // first upward and top first downward; one launch per depth and direction
  P.small_up.clear();
  P.small_down.clear();
  P.small_kids.clear();
  P.small_inv.clear();
  std::vector<int64_t> small_up_begin(P.n_levels + 1, 0), small_down_begin(P.n_levels + 1, 0);
  std::vector<double> small_fl_up(P.n_levels, 0.0), small_fl_down(P.n_levels, 0.0);
  {
    auto base = [&](int f) {
      const Front& F = P.fronts[f];
      SmallFront s{};
      s.panel_off = F.panel_off;
      s.l_off = F.l_off;
      s.upd_off = F.upd_off;
      s.asm_begin = asm_small_begin[f];
      s.asm_end = asm_small_end[f];
      s.rel_off = rel_off[f];
      s.nj = F.nj;
      s.nu = F.nu;
      s.depth = F.depth;
      s.parent_small = 0;
      if (F.parent >= 0) {
        const Front& Pa = P.fronts[F.parent];
        s.ppanel_off = Pa.panel_off;
        s.pguu_off = Pa.upd_off;
        s.pnj = Pa.nj;
        s.pnu = Pa.nu;
        s.parent_small = small[F.parent] ? 1 : 0;
      }
      return s;
    };
    // upward lists: small_up_begin[d] .. small_up_begin[d + 1] for depth d,
    // stored deepest first (the range of depth d starts after those deeper)
    for (int d = P.n_levels - 1; d >= 0; --d) {
      small_up_begin[d] = static_cast<int64_t>(P.small_up.size());
      for (int f : by_depth[d]) {
        if (!small[f]) continue;
        const Front& F = P.fronts[f];
        SmallFront s = base(f);
        s.child_begin = static_cast<int32_t>(P.small_kids.size());
        s.child_count = static_cast<int32_t>(F.children.size());
        for (int c : F.children) {
          const Front& C = P.fronts[c];
          std::vector<int32_t> inv(F.nj + F.nu, -1);
          for (int k = 0; k < C.nu; ++k) inv[C.rel[k]] = k;
          P.small_kids.push_back(SmallChild{C.upd_off, static_cast<int64_t>(P.small_inv.size()), C.nu, 0});
          P.small_inv.insert(P.small_inv.end(), inv.begin(), inv.end());
        }
        P.small_up.push_back(s);
        const double fu = 8.0 * (double(F.nj) * F.nj * F.nj + double(F.nu) * F.nj * F.nj + double(F.nu) * F.nu * F.nj / 2);
        const double fd = 8.0 * (double(F.nu) * F.nu * F.nj + double(F.nu) * F.nj * F.nj / 2);
        small_fl_up[d] += fu;
        small_fl_down[d] += fd;
        P.flops_exec += fu + fd;
      }
    }
    small_up_begin[P.n_levels] = static_cast<int64_t>(P.small_up.size());
    for (int d = 0; d < P.n_levels; ++d) {
      small_down_begin[d] = static_cast<int64_t>(P.small_down.size());
      for (int f : by_depth[d])
        if (small[f]) P.small_down.push_back(base(f));
    }
    small_down_begin[P.n_levels] = static_cast<int64_t>(P.small_down.size());
  }
  // the upward launch of the small fronts of depth d, then their downward one
  auto small_op = [&](int d, bool up) {
    Op op;
    op.kind = OP_SMALL;
    op.flags = up ? 0 : 1;
    if (up) {
      op.begin = small_up_begin[d];
      // the range of depth d ends where the next shallower depth's starts
      op.count = (d > 0 ? small_up_begin[d - 1] : small_up_begin[P.n_levels]) - op.begin;
      op.flops = small_fl_up[d];
    } else {
      op.begin = small_down_begin[d];
      op.count = small_down_begin[d + 1] - op.begin;
      op.flops = small_fl_down[d];
    }
    op.depth = d;
    return op;
  };

  // ---- program
  Builder B(P);
  const int64_t kTile = 1024;
  for (int d = P.n_levels - 1; d >= 0; --d) {
    {
      const Op op = small_op(d, true);
      if (op.count) P.upward.push_back(op);
    }
    std::vector<int> fr;
    for (int f : by_depth[d])
      if (!small[f]) fr.push_back(f);
    const int ubuf = (d % 2 == 0) ? BUF_UPD0 : BUF_UPD1;
    const int cbuf = (d % 2 == 0) ? BUF_UPD1 : BUF_UPD0;
    // extend-add into the panels (every element the pivot inverse and the
    // update GEMMs read); the U x U blocks take theirs in the epilogue of the
    // Schur-update GEMM below
    std::vector<int32_t> ext_index(P.fronts.size(), -1);
    {
      Op op;
      op.kind = OP_EXTADD;
      op.buf_a = cbuf, op.buf_b = ubuf, op.buf_c = BUF_PANEL;
      op.begin = static_cast<int64_t>(P.ext.size());
      op.tile_begin = static_cast<int64_t>(P.ext_tiles.size());
      op.depth = d;
      for (int f : fr) {
        const Front& F = P.fronts[f];
        ExtAddDesc ds{F.panel_off, F.upd_off, F.nj, F.nu, static_cast<int32_t>(P.ext_child.size()),
                      static_cast<int32_t>(F.children.size())};
        for (int c : F.children) {
          const Front& C = P.fronts[c];
          ExtAddChild ch{C.upd_off, static_cast<int64_t>(P.ext_inv.size()), C.nu, 0};
          std::vector<int32_t> inv(F.nj + F.nu, -1);
          for (int k = 0; k < C.nu; ++k) inv[C.rel[k]] = k;
          P.ext_inv.insert(P.ext_inv.end(), inv.begin(), inv.end());
          P.ext_child.push_back(ch);
        }
        const int32_t di = static_cast<int32_t>(P.ext.size() - op.begin);
        ext_index[f] = static_cast<int32_t>(P.ext.size());
        P.ext.push_back(ds);
        // tiles lying wholly above the diagonal 64 x 64 blocks of the pivot
        // block are left out (the extend-add skips those elements, below)
        const int64_t ld = F.nj + F.nu, total = ld * F.nj;
        for (int64_t e0 = 0; e0 < total; e0 += kTile) {
          const int64_t s0 = e0 / ld;
          if (e0 + kTile <= s0 * ld + 64 * (s0 / 64)) continue;
          P.ext_tiles.push_back(ElemTile{di, 0, e0});
        }
      }
      op.count = static_cast<int64_t>(P.ext.size()) - op.begin;
      op.tile_count = static_cast<int64_t>(P.ext_tiles.size()) - op.tile_begin;
      if (op.count) P.upward.push_back(op);
    }
    // assembly of alpha S - H into the panels of this depth
    if (P.asm_depth_begin[d + 1] > P.asm_depth_begin[d]) {
      Op op;
      op.kind = OP_ASSEMBLE;
      op.buf_c = BUF_PANEL;
      op.begin = P.asm_depth_begin[d];
      op.count = P.asm_depth_begin[d + 1] - P.asm_depth_begin[d];
      op.depth = d;
      P.upward.push_back(op);
    }
    // pivot-block inverses: blocks of <= 64 rows in one launch, larger ones
    // grouped by their number of 64-row blocks
    {
      std::vector<InvDesc> small;
      std::map<int, std::vector<int>> groups;
      for (int f : fr) {
        const Front& F = P.fronts[f];
        if (F.nj <= 64) small.push_back(InvDesc{F.panel_off, F.nj + F.nu, F.nj});
        else groups[(F.nj + 63) / 64].push_back(f);
      }
      B.smallinv(P.upward, small, d);
      for (auto& g : groups) {
        std::vector<int> nv, r0(g.second.size(), 0);
        std::vector<int64_t> t0(g.second.size(), 0);
        for (int f : g.second) nv.push_back(P.fronts[f].nj);
        B.inverse(P.upward, g.second, nv, r0, t0, d);
      }
    }
    // L = B A^{-1} (into the L buffer);  Upd = Upd - L B^T (lower triangle)
    {
      std::vector<GemmProb> g1, g2;
      for (int f : fr) {
        const Front& F = P.fronts[f];
        if (F.nu == 0) continue;
        const int ld = F.nj + F.nu;
        g1.push_back(GemmProb{F.nu, F.nj, F.nj, ld, ld, 0, F.nu, 0, F.panel_off + F.nj, F.panel_off, 0, F.l_off});
        g2.push_back(GemmProb{F.nu, F.nu, F.nj, F.nu, ld, 0, F.nu, ext_index[f], F.l_off, F.panel_off + F.nj, 0,
                              F.upd_off});
      }
      B.gemm(P.upward, 0, BUF_PANEL, BUF_PANEL, 0, BUF_L, g1, d);
      // C0 of the update is the children's extend-add, read from the deeper buffer
      B.gemm(P.upward, G_TB | G_SYM | G_EXTC0 | G_NEG | G_NOMIRROR, BUF_L, BUF_PANEL, cbuf, ubuf, g2, d);
    }
  }
  for (int d = 1; d < P.n_levels; ++d) {
    std::vector<int> fr, top;  // large fronts; small fronts with a large parent
    for (int f : by_depth[d]) {
      if (!small[f]) fr.push_back(f);
      else if (!small[P.fronts[f].parent]) top.push_back(f);
    }
    const int ubuf = (d % 2 == 0) ? BUF_UPD0 : BUF_UPD1;
    const int pbuf = (d % 2 == 0) ? BUF_UPD1 : BUF_UPD0;
    // G_UU of the small fronts whose parent is large, gathered here (right
    // after the parent's level) into their own blocks, kept FP64 for the
    // small-front launch of this depth that continues from them
    for (int pass = 0; pass < 2; ++pass) {
      const std::vector<int>& list = pass == 0 ? fr : top;
      Op op;
      op.kind = OP_GATHER;
      op.keep64 = pass == 1;
      op.buf_a = pbuf, op.buf_b = BUF_PANEL, op.buf_c = ubuf;
      op.begin = static_cast<int64_t>(P.gat.size());
      op.tile_begin = static_cast<int64_t>(P.gat_tiles.size());
      op.depth = d;
      for (int f : list) {
        const Front& F = P.fronts[f];
        if (F.nu == 0) continue;
        const Front& Pa = P.fronts[F.parent];
        const int32_t di = static_cast<int32_t>(P.gat.size() - op.begin);
        P.gat.push_back(GatherDesc{F.upd_off, rel_off[f], Pa.panel_off, Pa.upd_off, F.nu, Pa.nj, Pa.nu, 0});
        // G_UU is kept as its lower triangle: tiles wholly above it are left out
        const int64_t total = int64_t(F.nu) * F.nu;
        for (int64_t e0 = 0; e0 < total; e0 += kTile) {
          const int64_t b0 = e0 / F.nu;
          if (e0 + kTile <= b0 * (F.nu + 1)) continue;
          P.gat_tiles.push_back(ElemTile{di, 0, e0});
        }
      }
      op.count = static_cast<int64_t>(P.gat.size()) - op.begin;
      op.tile_count = static_cast<int64_t>(P.gat_tiles.size()) - op.tile_begin;
      if (op.count) P.downward.push_back(op);
    }
    std::vector<GemmProb> g3, g4;
    for (int f : fr) {
      const Front& F = P.fronts[f];
      if (F.nu == 0) continue;
      const int ld = F.nj + F.nu;
      // G_UJ = -G_UU L, written over B in the panel (G_UU from its lower triangle)
      g3.push_back(GemmProb{F.nu, F.nj, F.nu, F.nu, F.nu, 0, ld, 0, F.upd_off, F.l_off, 0, F.panel_off + F.nj});
      // G_JJ = A^{-1} - L^T G_UJ
      g4.push_back(GemmProb{F.nj, F.nj, F.nu, F.nu, ld, ld, ld, 0, F.l_off, F.panel_off + F.nj, F.panel_off,
                            F.panel_off});
    }
    B.gemm(P.downward, G_NEG | G_SYMA, ubuf, BUF_L, 0, BUF_PANEL, g3, d);
    B.gemm(P.downward, G_TA | G_SYM | G_BETA | G_NEG, BUF_L, BUF_PANEL, BUF_PANEL, BUF_PANEL, g4, d);
    {
      const Op op = small_op(d, false);
      if (op.count) P.downward.push_back(op);
    }
  }
}

void join_plans(Plan& U, const std::vector<const Plan*>& parts) {
  U = Plan();
  int64_t rows = 0, nnz = 0;
  int levels = 0;
  U.row_ptr.push_back(0);
  for (const Plan* p : parts) {
    const int fbase = static_cast<int>(U.fronts.size());
    U.struct_row_off.push_back(rows);
    U.struct_nnz_off.push_back(nnz);
    for (int64_t i = 0; i < p->n; ++i) U.row_ptr.push_back(nnz + p->row_ptr[i + 1]);
    for (int64_t e = 0; e < p->nnz; ++e) U.col.push_back(static_cast<int32_t>(p->col[e] + rows));
    for (int64_t i = 0; i < p->n; ++i) {
      U.perm.push_back(static_cast<int32_t>(p->perm[i] + rows));
      U.iperm.push_back(static_cast<int32_t>(p->iperm[i] + rows));
    }
    for (const Front& F0 : p->fronts) {
      Front F = F0;
      if (F.parent >= 0) F.parent += fbase;
      for (int& c : F.children) c += fbase;
      F.j0 += rows;
      for (int& q : F.u) q += static_cast<int>(rows);
      U.fronts.push_back(std::move(F));
    }
    rows += p->n;
    nnz += p->nnz;
    levels = std::max(levels, p->n_levels);
  }
  U.n = rows;
  U.nnz = nnz;
  U.n_levels = levels;
  U.small_enabled = parts.empty() ? true : parts[0]->small_enabled;
  finalize_plan(U);
}

}  // namespace ndrho
