// C interface of the ndrho library: contexts, structures, poles, and the
// executor that replays a structure's launch program for each pole batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"
#include "plan.h"

using namespace ndrho;

namespace {

#define HIP_OK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) fail(NDRHO_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
T* upload(const std::vector<T>& v, hipStream_t st) {
  if (v.empty()) return nullptr;
  T* p = nullptr;
  if (hipMalloc(&p, v.size() * sizeof(T)) != hipSuccess) fail(NDRHO_ENOMEM, "device allocation failed");
  HIP_OK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return p;
}

struct DevStruct {
  Plan plan;
  int32_t split_passes = 0;  // passes of the last recorded evaluation run as several chains
  std::vector<void*> allocs;
  double *h = nullptr, *s = nullptr, *m0 = nullptr;
  // first moment of G, S^-1 H S^-1 on the pattern (computed on first use)
  double* m1 = nullptr;
  bool m1_valid = false;
  double h_inf = 0.0;  // max_i sum_j |H_ij|
  GemmProb* gemm = nullptr;
  TileRef* gemm_tiles = nullptr;
  InvDesc* inv = nullptr;
  CopyDesc* copy = nullptr;
  CopyTile* copy_tiles = nullptr;
  ExtAddDesc* ext = nullptr;
  ExtAddChild* ext_child = nullptr;
  int32_t* ext_inv = nullptr;
  ElemTile *ext_tiles = nullptr, *gat_tiles = nullptr;
  GatherDesc* gat = nullptr;
  int32_t* rel = nullptr;
  int64_t* asm_slot = nullptr;
  int32_t* asm_entry = nullptr;
  int32_t* asm_sid = nullptr;
  int64_t* acc_slot = nullptr;
  int32_t* acc_entry = nullptr;
  int32_t* acc_sid = nullptr;  // joined plans: structure of each sorted pattern slot
  SmallFront *small_up = nullptr, *small_down = nullptr;  // the fused small-front launches' fronts
  SmallChild* small_kids = nullptr;
  int32_t* small_inv = nullptr;
  // shifts and weights
  int n_shifts = 0;
  int n_hi = 0;  // leading shifts evaluated with FP64 front updates
  bool add_m0 = true;
  bool cf_poles = false;  // shifts are the continued-fraction poles of set_poles
  double kappa = 0.0;     // (4/beta) sum_p R_p = -sum_p w_p (Eq. (11))
  double2* d_alpha = nullptr;
  double* d_w = nullptr;
  double2* d_cw = nullptr;  // w_p alpha_p, the weights of the energy density matrix
  std::vector<double> w_host;  // weights as set (batch compatibility checks)
  std::vector<double> s_host;  // S in CSR order (electron count Tr(rho S))
  std::vector<double> h_host;  // H in CSR order
  // GEMM variant per program op (empty: default heuristic not yet applied)
  std::vector<int8_t> variant;
  int tune_gen = 0;
  // captured launch sequence of a full evaluation, valid for `gkey`
  hipGraphExec_t gexec = nullptr;
  std::vector<const void*> gkey;
  // solves through the stored factor (selected eigenstates), built on first use
  struct EigenPlan {
    bool built = false;
    SolveFront* fronts = nullptr;
    SolveChild* kids = nullptr;
    int32_t *inv = nullptr, *urows = nullptr, *perm = nullptr, *iperm = nullptr, *col = nullptr;
    int64_t* rp = nullptr;
    SolveTile* gtiles = nullptr;
    TsProb* probs = nullptr;
    TsTile* ttiles = nullptr;
    int64_t w_rows = 0;
    // per depth: forward-gather tiles, forward / backward product tiles; one range for the diagonal
    std::vector<int64_t> g_begin, f_begin, b_begin;
    int64_t d_begin = 0, d_count = 0;
  } eig;

  template <class T>
  T* put(const std::vector<T>& v, hipStream_t st) {
    T* p = upload(v, st);
    if (p) allocs.push_back(p);
    return p;
  }
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
    gkey.clear();
  }
  void release() {
    drop_graph();
    for (void* p : allocs) (void)hipFree(p);
    allocs.clear();
    if (d_alpha) (void)hipFree(d_alpha);
    if (d_w) (void)hipFree(d_w);
    if (d_cw) (void)hipFree(d_cw);
    d_alpha = nullptr;
    d_w = nullptr;
    d_cw = nullptr;
  }
};

thread_local std::string g_err;  // errors without a context (create, plan utilities)

// Fixed device scratch of the no-allocation entry point
// (ndrho_density_matrix_noalloc): the pole workspace, the pole-sum
// accumulator and the pivot status words of one call live here instead of in
// allocations.  Each device holds its own copy at its own address, looked up
// once per device (hipGetSymbolAddress) and kept in scratch_addr; host code
// passes only that address to kernels and copies, never the symbol itself.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) double2 scratch[kScratchBytes / sizeof(double2)];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Address of this device's scratch (the device must be current); looked up
// on the first call for the device.
void* scratch_addr(int device) {
  if (device < 0 || device >= kMaxDevices) fail(NDRHO_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      fail(NDRHO_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_addr[device] = p;
  }
  return g_scratch_addr[device];
}

// max_i sum_j |A_ij| of a matrix on the plan's pattern (values in CSR order)
double row_sum_norm(const Plan& P, const double* a) {
  double mx = 0.0;
  for (int64_t i = 0; i < P.n; ++i) {
    double r = 0.0;
    for (int64_t k = P.row_ptr[i]; k < P.row_ptr[i + 1]; ++k) r += std::fabs(a[k]);
    mx = std::max(mx, r);
  }
  return mx;
}

enum { V_FP64 = 0, V_F32_64 = 1, V_F32_128 = 2, V_BF3_128 = 3, V_BF3_64 = 4, V_BF3S_128 = 5, V_BF3P_128 = 6, V_BF3W_128 = 7,
       V_COUNT = 8 };

// Variants a precision mode may choose from: FP32 mode its FP32 products;
// split-BF16 mode its split-BF16 products and, where a launch runs faster
// so, FP32 products (the two have the same operand rounding and accuracy).
static bool variant_allowed(int precision, int v) {
  if (v == V_FP64) return true;
  if (precision == NDRHO_MIXED_FP32) return v == V_F32_64 || v == V_F32_128;
  if (precision == NDRHO_MIXED_BF16X3) return v != V_FP64;
  return false;
}

// Default GEMM variant per op before any tuning: low-precision products on
// 128x128 tiles (front updates) or 64x64 tiles (the pivot-block inverse's
// products) where the op's largest problem fills several such tiles, plain
// FP64 for the small fronts of the deep levels (where they do not pay).
std::vector<int8_t> default_variants(const Plan& P, int precision) {
  const int8_t low = precision == NDRHO_MIXED_BF16X3 ? int8_t(V_BF3_128) : int8_t(V_F32_128);
  const int8_t low_piv = precision == NDRHO_MIXED_BF16X3 ? int8_t(V_BF3_64) : int8_t(V_F32_64);
  std::vector<int8_t> v;
  auto pick = [&](const Op& op) {
    if (op.kind != OP_GEMM) return int8_t(V_FP64);
    int mx = 0;
    for (int64_t i = 0; i < op.count; ++i) {
      const GemmProb& g = P.gemm[op.begin + i];
      mx = std::max(mx, std::min(g.m, g.n));
    }
    if (mx < 256) return int8_t(V_FP64);
    return (op.flags & OP_PIVOT) ? low_piv : low;
  };
  for (const Op& op : P.upward) v.push_back(pick(op));
  for (const Op& op : P.downward) v.push_back(pick(op));
  return v;
}

// Device copies of a plan's descriptor arrays and tables.
void upload_plan(DevStruct& ds, hipStream_t st, int precision) {
  const Plan& P = ds.plan;
  ds.gemm = ds.put(P.gemm, st);
  ds.gemm_tiles = ds.put(P.gemm_tiles, st);
  ds.inv = ds.put(P.inv, st);
  ds.copy = ds.put(P.copy, st);
  ds.copy_tiles = ds.put(P.copy_tiles, st);
  ds.ext = ds.put(P.ext, st);
  ds.ext_child = ds.put(P.ext_child, st);
  ds.ext_inv = ds.put(P.ext_inv, st);
  ds.ext_tiles = ds.put(P.ext_tiles, st);
  ds.gat = ds.put(P.gat, st);
  ds.gat_tiles = ds.put(P.gat_tiles, st);
  ds.rel = ds.put(P.rel_all, st);
  ds.asm_slot = ds.put(P.asm_slot_sorted, st);
  ds.asm_entry = ds.put(P.asm_entry_sorted, st);
  ds.asm_sid = ds.put(P.asm_sid_sorted, st);
  ds.acc_slot = ds.put(P.acc_slot, st);
  ds.acc_entry = ds.put(P.acc_entry, st);
  ds.small_up = ds.put(P.small_up, st);
  ds.small_down = ds.put(P.small_down, st);
  ds.small_kids = ds.put(P.small_kids, st);
  ds.small_inv = ds.put(P.small_inv, st);
  ds.variant = default_variants(P, precision);
}

}  // namespace

struct ndrho_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // further streams of a split pass (FP64 poles and parts of the
  // low-precision ones beside `stream`), the event that forks them from
  // `stream` and one per stream that joins it back
  static constexpr int kMaxChains = 4;
  hipStream_t side[kMaxChains] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kMaxChains] = {};
  ndrho_options opt{};
  std::string err;
  std::vector<std::unique_ptr<DevStruct>> structs;
  // joined plans of structure batches, keyed by the list of structure ids
  std::map<std::vector<int32_t>, std::unique_ptr<DevStruct>> unions;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  double* acc = nullptr;
  double* outbuf = nullptr;
  int64_t acc_len = 0;
  // energy density matrix accumulator and output staging (allocated on first use)
  double* acc_e = nullptr;
  double* outbuf_e = nullptr;
  int64_t acc_e_len = 0;
  int* status = nullptr;  // [0] singular pivots, [1] non-positive pivots of S, [2], [3] spare
  void* scratch = nullptr;  // this device's fixed scratch (no-allocation entry point)
  double last_ms = 0;
  int last_batch = 0;
  // profiling: events around launches, folded into per-kind totals
  bool prof = false;
  std::vector<hipEvent_t> events;
  struct Rec {
    int kind;
    size_t ev;
    double flops;
    double bytes;
    int op;  // program index of the launch (upward ops, then downward), -1 for the pole sum
    int depth;
    int phase;
  };
  int cur_op = -1;
  int cur_depth = -1;
  int cur_phase = 3;  // 0 assembly, 1 upward sweep, 2 downward sweep, 3 pole sum and the rest
  std::vector<double>* op_ms = nullptr;  // per-op milliseconds while autotuning
  std::vector<Rec> recs;
  double prof_ms[NDRHO_K_COUNT] = {0};
  double prof_flops[NDRHO_K_COUNT] = {0};
  double prof_bytes[NDRHO_K_COUNT] = {0};
  int64_t prof_n[NDRHO_K_COUNT] = {0};
  double prof_depth_ms[NDRHO_K_COUNT * NDRHO_PROFILE_DEPTHS] = {0};
  double prof_phase_ms[4] = {0};
  // algorithmic flops and bytes (the plan's model) of the last evaluation
  double last_flops = 0, last_bytes = 0;
  void clear_profile() {
    for (int k = 0; k < NDRHO_K_COUNT; ++k) prof_ms[k] = prof_flops[k] = prof_bytes[k] = 0, prof_n[k] = 0;
    for (double& x : prof_depth_ms) x = 0;
    for (double& x : prof_phase_ms) x = 0;
  }

  hipEvent_t event(size_t i) {
    while (events.size() <= i) {
      hipEvent_t e;
      HIP_OK(hipEventCreate(&e));
      events.push_back(e);
    }
    return events[i];
  }
  // bracket a launch when profiling
  template <class L>
  void timed(int kind, double flops, L&& launch, double bytes = 0.0) {
    if (!prof) {
      launch();
      return;
    }
    const size_t i = 2 * recs.size();
    HIP_OK(hipEventRecord(event(i), stream));
    launch();
    HIP_OK(hipEventRecord(event(i + 1), stream));
    recs.push_back(Rec{kind, i, flops, bytes, cur_op, cur_depth, kind == NDRHO_K_ASSEMBLE ? 0 : cur_phase});
  }
  // fold recorded events into the totals (stream must be complete)
  void fold_profile() {
    for (const Rec& r : recs) {
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, events[r.ev], events[r.ev + 1]));
      prof_ms[r.kind] += ms;
      prof_flops[r.kind] += r.flops;
      prof_bytes[r.kind] += r.bytes;
      prof_n[r.kind] += 1;
      prof_phase_ms[r.phase] += ms;
      const int d = r.depth < 0 ? NDRHO_PROFILE_DEPTHS - 1 : std::min(r.depth, NDRHO_PROFILE_DEPTHS - 2);
      prof_depth_ms[r.kind * NDRHO_PROFILE_DEPTHS + d] += ms;
      if (op_ms && r.op >= 0 && r.op < static_cast<int>(op_ms->size())) (*op_ms)[r.op] += ms;
    }
    recs.clear();
  }

  ~ndrho_ctx() {
    // Teardown order: the streams' work completes, the captured graphs go,
    // the device drains, the further streams and events go, and only then is
    // memory freed (memory that a graph with forked streams ran on was
    // otherwise kept by the runtime after hipFree).
    if (stream) (void)hipStreamSynchronize(stream);
    for (int i = 0; i < kMaxChains; ++i)
      if (side[i]) (void)hipStreamSynchronize(side[i]);
    for (auto& s : structs)
      if (s) s->drop_graph();
    for (auto& u : unions) u.second->drop_graph();
    (void)hipDeviceSynchronize();
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    for (int i = 0; i < kMaxChains; ++i) {
      if (ev_join[i]) (void)hipEventDestroy(ev_join[i]);
      if (side[i]) (void)hipStreamDestroy(side[i]);
    }
    for (auto& s : structs)
      if (s) s->release();
    for (auto& u : unions) u.second->release();
    if (ws) (void)hipFree(ws);
    if (acc) (void)hipFree(acc);
    if (outbuf) (void)hipFree(outbuf);
    if (acc_e) (void)hipFree(acc_e);
    if (outbuf_e) (void)hipFree(outbuf_e);
    if (status) (void)hipFree(status);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }

  DevStruct& get(int32_t id) {
    if (id < 0 || id >= static_cast<int32_t>(structs.size()) || !structs[id])
      fail(NDRHO_EINVAL, "invalid struct_id");
    return *structs[id];
  }

  // complex elements per pole of the workspace
  static int64_t per_pole_elems(const Plan& P) {
    return P.panel_total + 2 * P.upd_total + P.temp_total + P.l_total;
  }

  // Workspace for `nb` poles of plan P (grown, never shrunk).
  void ensure_ws(const Plan& P, int nb) {
    const size_t need = static_cast<size_t>(per_pole_elems(P)) * nb * sizeof(double2);
    if (need > ws_bytes) {
      if (ws) {
        // graphs captured on the old workspace go first (their keys hold its
        // address, so they would be captured again anyway)
        HIP_OK(hipStreamSynchronize(stream));
        for (int i = 0; i < kMaxChains; ++i)
          if (side[i]) HIP_OK(hipStreamSynchronize(side[i]));
        for (auto& s : structs)
          if (s) s->drop_graph();
        for (auto& u : unions) u.second->drop_graph();
        HIP_OK(hipDeviceSynchronize());
        HIP_OK(hipFree(ws));
      }
      ws = nullptr;
      ws_bytes = 0;
      if (hipMalloc(&ws, need) != hipSuccess) {
        (void)hipGetLastError();
        fail(NDRHO_ENOMEM, "workspace allocation of " + std::to_string(need) + " bytes failed");
      }
      ws_bytes = need;
    }
    if (P.nnz > acc_len) {
      if (acc) HIP_OK(hipFree(acc));
      if (outbuf) HIP_OK(hipFree(outbuf));
      acc = outbuf = nullptr;
      if (hipMalloc(&acc, P.nnz * sizeof(double)) != hipSuccess ||
          hipMalloc(&outbuf, P.nnz * sizeof(double)) != hipSuccess)
        fail(NDRHO_ENOMEM, "accumulator allocation failed");
      acc_len = P.nnz;
    }
  }

  // Poles per device pass for plan P.
  int batch_for(const Plan& P, int n_shifts) {
    if (opt.pole_batch > 0) return std::min(opt.pole_batch, n_shifts);
    size_t free_b = 0, total_b = 0;
    HIP_OK(hipMemGetInfo(&free_b, &total_b));
    const double budget = opt.mem_fraction * (static_cast<double>(free_b) + static_cast<double>(ws_bytes));
    const double pp = static_cast<double>(per_pole_elems(P)) * sizeof(double2);
    const double fit = std::floor(budget / pp);  // may exceed the int range for tiny plans
    if (fit < 1.0) fail(NDRHO_ENOMEM, "one pole needs " + std::to_string(pp) + " bytes; budget " + std::to_string(budget));
    return fit >= static_cast<double>(n_shifts) ? n_shifts : static_cast<int>(fit);
  }

  // Workspace regions of a batch of `nlay` poles: each buffer kind holds
  // its poles one after another, `strides` elements apart.
  void layout(const Plan& P, int nlay, double2** bufs, int64_t* strides) const {
    double2* base = static_cast<double2*>(ws);
    bufs[BUF_PANEL] = base;
    strides[BUF_PANEL] = P.panel_total;
    bufs[BUF_UPD0] = base + P.panel_total * nlay;
    strides[BUF_UPD0] = P.upd_total;
    bufs[BUF_UPD1] = bufs[BUF_UPD0] + P.upd_total * nlay;
    strides[BUF_UPD1] = P.upd_total;
    bufs[BUF_TEMP] = bufs[BUF_UPD1] + P.upd_total * nlay;
    strides[BUF_TEMP] = P.temp_total;
    bufs[BUF_L] = bufs[BUF_TEMP] + P.temp_total * nlay;
    strides[BUF_L] = P.l_total;
  }

  // One pass of the whole program (assembly, upward and downward sweeps;
  // the pole sum is left to the caller) over `nb` poles held at positions
  // q0 .. q0 + nb - 1 of a workspace laid out for `nlay` poles, launched on
  // `st`; the first `nhi` of them take FP64 front updates, the rest the
  // context's low precision (pivot inverses are FP64 for all).  Passes over
  // disjoint position ranges share no memory but the pivot status counters,
  // which are updated atomically.
  void run_pass(DevStruct& S, int nlay, int q0, int nb, const double2* alpha, int64_t astride, double hcoef,
                int spd_check, int nhi, hipStream_t st, bool up_only = false) {
    const Plan& P = S.plan;
    double2* bufs[BUF_COUNT];
    int64_t strides[BUF_COUNT];
    layout(P, nlay, bufs, strides);
    for (int b = 0; b < BUF_COUNT; ++b) bufs[b] += q0 * strides[b];
    auto resolve = [&](const Op& op) {
      DevOp d;
      d.flags = op.flags & 0xff;
      d.npoles = nb;
      d.count = op.count;
      d.tile_count = op.tile_count;
      d.a = bufs[op.buf_a], d.sa = strides[op.buf_a];
      d.b = bufs[op.buf_b], d.sb = strides[op.buf_b];
      d.c0 = bufs[op.buf_c0], d.sc0 = strides[op.buf_c0];
      d.c = bufs[op.buf_c], d.sc = strides[op.buf_c];
      return d;
    };
    // G_UU of the low-precision poles is kept as FP32 complex at the depths
    // where its only consumer, the G_UJ = -G_UU L launch, runs those poles in
    // low precision (its products round the operand to FP32 in any case)
    std::vector<char> guu32(P.n_levels + 1, 0);
    for (size_t i = 0; i < P.downward.size(); ++i) {
      const Op& op = P.downward[i];
      if (op.kind != OP_GEMM || op.flags != (G_NEG | G_SYMA)) continue;
      const int var = opt.gemm_variant >= 0 ? opt.gemm_variant : S.variant[P.upward.size() + i];
      guu32[op.depth] = nhi < nb && var != V_FP64;
    }
    auto run = [&](const Op& op) {
      DevOp d = resolve(op);
      hipError_t e = hipSuccess;
      switch (op.kind) {
        case OP_EXTADD:
          d.ext = S.ext + op.begin;
          d.ext_child = S.ext_child;
          d.ext_inv = S.ext_inv;
          d.elem_tiles = S.ext_tiles + op.tile_begin;
          timed(NDRHO_K_EXTADD, 0.0, [&] { e = launch_extadd(d, st); });
          break;
        case OP_ASSEMBLE:
          d.slot = S.asm_slot + op.begin;
          d.entry = S.asm_entry + op.begin;
          d.sid = S.asm_sid + op.begin;
          timed(NDRHO_K_ASSEMBLE, 0.0, [&] { e = launch_assemble(d, S.h, S.s, alpha, astride, hcoef, st); });
          break;
        case OP_SMALLINV:
          d.inv = S.inv + op.begin;
          d.count16 = op.inv16;
          d.count32 = op.inv32;
          timed(NDRHO_K_PIVOT_INV, 0.0, [&] { e = launch_smallinv(d, status, spd_check, st); });
          break;
        case OP_GEMM: {
          d.gemm = S.gemm + op.begin;
          d.ext = S.ext;  // G_EXTC0: the children of each problem's front
          d.ext_child = S.ext_child;
          d.ext_inv = S.ext_inv;
          d.gemm_tiles = S.gemm_tiles + op.tile_begin;
          // variant of a front-update GEMM (chosen by heuristic or by the
          // autotuner, or forced by gemm_variant): V_FP64 keeps every pole in
          // FP64; the others give the low poles FP32 products (V_F32_64,
          // V_F32_128) or split-BF16 products (V_BF3_128, V_BF3_64, V_BF3S_128, V_BF3P_128,
          // V_BF3W_128)
          // (pivot-inverse GEMMs: pivot_variant if set, else the per-launch choice)
          const bool pivot = (op.flags & OP_PIVOT) != 0;
          const int forced = pivot ? opt.pivot_variant : opt.gemm_variant;
          int var = forced >= 0 ? forced : S.variant[cur_op];
          if ((var == V_BF3P_128 || var == V_BF3W_128) && !op.off32) var = V_BF3_128;  // 32-bit operand offsets only
          const bool split = nhi < nb && var != V_FP64;
          const int k64 = (op.flags & OP_PIVOT) ? NDRHO_K_GEMM_PIVOT : NDRHO_K_GEMM;
          // FP64 launches of small problems: two waves per 32x32 tile, no LDS
          const bool small = opt.fp64_small_tiles < 0 ? op.small : opt.fp64_small_tiles != 0;
          auto fp64_launch = [&](DevOp x) {
            if (small) {
              x.small = true;
              x.gemm_tiles = S.gemm_tiles + op.tile32_begin;
              x.tile_count = op.tile32_count;
            }
            return x;
          };
          if (!split) {
            const DevOp h = fp64_launch(d);
            timed(k64, op.flops * nb, [&] { e = launch_gemm(h, st); }, op.bytes * nb);
            break;
          }
          if (nhi > 0) {  // FP64 for the poles nearest the real axis
            DevOp h = fp64_launch(d);
            h.npoles = nhi;
            timed(k64, op.flops * nhi, [&] { e = launch_gemm(h, st); }, op.bytes * nhi);
            if (e != hipSuccess) break;
          }
          DevOp l = d;  // low-precision products for the others
          l.fp32 = var == V_F32_64 || var == V_F32_128;
          l.bf3 = var == V_BF3_128 ? 1 : var == V_BF3_64 ? 2 : var == V_BF3S_128 ? 3 : var == V_BF3P_128 ? 4
                 : var == V_BF3W_128 ? 5 : 0;
          if (var == V_F32_128 || var == V_BF3_128 || var == V_BF3S_128 || var == V_BF3P_128 || var == V_BF3W_128) {
            l.tile128 = true;
            l.gemm_tiles = S.gemm_tiles + op.tile128_begin;
            l.tile_count = op.tile128_count;
          }
          l.npoles = nb - nhi;
          l.a32 = op.flags == (G_NEG | G_SYMA) && guu32[op.depth];
          l.a += nhi * l.sa, l.b += nhi * l.sb, l.c += nhi * l.sc;
          if (op.flags & (G_BETA | G_EXTC0)) l.c0 += nhi * l.sc0;
          timed(pivot ? NDRHO_K_GEMM_PIVOT : l.bf3 ? NDRHO_K_GEMM_BF16X3 : NDRHO_K_GEMM_F32, op.flops * (nb - nhi),
                [&] { e = launch_gemm(l, st); }, op.bytes * (nb - nhi));
          break;
        }
        case OP_COPY:
          d.copy = S.copy + op.begin;
          d.copy_tiles = S.copy_tiles + op.tile_begin;
          timed(NDRHO_K_COPY, 0.0, [&] { e = launch_copy(d, st); });
          break;
        case OP_SMALL: {
          SmallLaunch sl;
          sl.up = op.flags == 0;
          sl.fronts = (sl.up ? S.small_up : S.small_down) + op.begin;
          sl.kids = S.small_kids;
          sl.inv = S.small_inv;
          sl.rel = S.rel;
          sl.nfronts = op.count;
          sl.npoles = nb;
          sl.panel = bufs[BUF_PANEL], sl.ps = strides[BUF_PANEL];
          sl.lbuf = bufs[BUF_L], sl.ls = strides[BUF_L];
          sl.upd0 = bufs[BUF_UPD0], sl.upd1 = bufs[BUF_UPD1], sl.us = strides[BUF_UPD0];
          sl.asm_slot = S.asm_slot, sl.asm_entry = S.asm_entry, sl.asm_sid = S.asm_sid;
          sl.hv = S.h, sl.sv = S.s;
          sl.alpha = alpha, sl.astride = astride, sl.hcoef = hcoef, sl.spd_check = spd_check;
          sl.status = status;
          timed(NDRHO_K_SMALL, op.flops * nb, [&] { e = launch_small(sl, st); });
          break;
        }
        case OP_GATHER:
          d.gat = S.gat + op.begin;
          d.rel = S.rel;
          d.elem_tiles = S.gat_tiles + op.tile_begin;
          d.nhi = nhi;
          d.gat_out32 = op.keep64 ? 0 : guu32[op.depth];
          d.gat_in32 = op.depth > 0 ? guu32[op.depth - 1] : 0;
          timed(NDRHO_K_GATHER, 0.0, [&] { e = launch_gather(d, st); });
          break;
      }
      if (e != hipSuccess) fail(NDRHO_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    };
    cur_op = 0;
    cur_phase = 1;
    for (const Op& op : P.upward) {
      cur_depth = op.depth;
      run(op);
      ++cur_op;
    }
    cur_phase = 2;
    for (const Op& op : P.downward) {
      if (up_only) break;
      cur_depth = op.depth;
      run(op);
      ++cur_op;
    }
    cur_op = -1;
    cur_depth = -1;
    cur_phase = 3;
  }

  // Passes of less work than this run as one chain: there the fork and join
  // cost more than the chains overlap (measured: 0.1 ms lost on a 256-site
  // chain with 4 orbitals per site and 60 poles, 5e8 flops per pass; 1.4 ms
  // gained on a 64 x 64-site square lattice with 4 orbitals, 3e11 flops).
  static constexpr double kSplitMinFlops = 1e10;

  // Create the first `k` further streams and their events on first use.
  void ensure_side(int k) {
    if (!ev_fork) HIP_OK(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
    for (int i = 0; i < k; ++i) {
      if (side[i]) continue;
      HIP_OK(hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking));
      HIP_OK(hipEventCreateWithFlags(&ev_join[i], hipEventDisableTiming));
    }
  }

  // Full weighted sum over the structure's shifts into `acc` (sorted order).
  // The first n_hi shifts run with FP64 front updates, the rest in the
  // context's low precision; the sum is taken in shift order either way.
  // With `edm`, the energy density matrix of the same shifts is summed
  // beside rho into acc_e: M1 + kappa M0 + sum_p Re(c_p G_p), c_p = S.d_cw.
  void evaluate(DevStruct& S, const double2* alpha, int64_t astride, const double* w, int n, int n_hi, bool add_m0,
                double hcoef, int spd_check, bool edm = false, double2* trace_partial = nullptr, int trace_nblk = 0) {
    const Plan& P = S.plan;
    const int nb = batch_for(P, n);
    ensure_ws(P, nb);
    last_batch = nb;
    last_flops = P.flops_model * n;
    last_bytes = P.bytes_model * n;
    auto record = [&] {
      HIP_OK(launch_init_acc(S.m0, P.nnz, add_m0 ? 1 : 0, acc, status, stream));
      if (edm) HIP_OK(launch_init_edm(S.m1, S.m0, S.kappa, P.nnz, acc_e, stream));
      S.split_passes = 0;
      // With several passes and both kinds of poles, every pass takes its
      // share of the FP64 poles (sorted first, [0, n_hi)) beside its share
      // of the low-precision ones, so that each pass can run as two chains;
      // within a pass, positions [0, nhi) hold the FP64 poles.
      const int npass = (n + nb - 1) / nb;
      const bool spread = npass > 1 && n_hi > 0 && n_hi < n;
      int c0 = 0, h0 = 0;  // poles, and FP64 poles, before this pass
      for (int b = 0; b < npass; ++b) {
        const int cnt = std::min(nb, n - c0);
        int nhi, hfirst, lfirst;  // FP64 count; indices of the first FP64 and first low pole
        if (spread) {
          const int h1 = static_cast<int>(int64_t(n_hi) * (c0 + cnt) / n);
          nhi = h1 - h0;
          hfirst = h0;
          lfirst = n_hi + (c0 - h0);
          h0 = h1;
        } else {
          nhi = std::max(0, std::min(cnt, n_hi - c0));
          hfirst = c0;
          lfirst = c0 + nhi;
        }
        c0 += cnt;
        const bool both = nhi > 0 && nhi < cnt;
        if (opt.split_streams > 0 && !prof && both && P.flops_exec * cnt >= kSplitMinFlops) {
          // the FP64 poles and the low-precision poles (in split_streams
          // parts) as independent launch chains: launches that leave compute
          // units idle (small fronts, memory-bound steps) overlap work of the
          // other chains
          const int parts = std::min(opt.split_streams, cnt - nhi);
          ++S.split_passes;
          ensure_side(parts);
          HIP_OK(hipEventRecord(ev_fork, stream));
          for (int i = 0; i < parts; ++i) HIP_OK(hipStreamWaitEvent(side[i], ev_fork, 0));
          run_pass(S, cnt, 0, nhi, alpha + hfirst, astride, hcoef, spd_check, nhi, side[0]);
          for (int i = 0; i < parts; ++i) {
            const int q0 = nhi + static_cast<int>(int64_t(cnt - nhi) * i / parts);
            const int q1 = nhi + static_cast<int>(int64_t(cnt - nhi) * (i + 1) / parts);
            run_pass(S, cnt, q0, q1 - q0, alpha + lfirst + (q0 - nhi), astride, hcoef, spd_check, 0,
                     i == 0 ? stream : side[i]);
          }
          for (int i = 0; i < parts; ++i) {
            HIP_OK(hipEventRecord(ev_join[i], side[i]));
            HIP_OK(hipStreamWaitEvent(stream, ev_join[i], 0));
          }
        } else if (both && lfirst != hfirst + nhi) {
          // the two ranges one after the other on one chain
          run_pass(S, cnt, 0, nhi, alpha + hfirst, astride, hcoef, spd_check, nhi, stream);
          run_pass(S, cnt, nhi, cnt - nhi, alpha + lfirst, astride, hcoef, spd_check, 0, stream);
        } else {
          run_pass(S, cnt, 0, cnt, alpha + (nhi > 0 ? hfirst : lfirst), astride, hcoef, spd_check, nhi, stream);
        }
        // pole sums over the pass: the FP64 positions, then the others
        double2* bufs[BUF_COUNT];
        int64_t strides[BUF_COUNT];
        layout(P, cnt, bufs, strides);
        auto sum_range = [&](int q0, int m, int first) {
          if (m <= 0) return;
          const double2* panel = bufs[BUF_PANEL] + int64_t(q0) * P.panel_total;
          hipError_t ea = hipSuccess;
          timed(NDRHO_K_ACCUM, 0.0,
                [&] { ea = launch_accum(S.acc_slot, P.nnz, panel, P.panel_total, w + first, m, acc, stream); });
          HIP_OK(ea);
          if (edm)
            timed(NDRHO_K_ACCUM, 0.0, [&] {
              ea = launch_accum_edm(S.acc_slot, P.nnz, panel, P.panel_total, S.d_cw + first, m, S.acc_sid, astride,
                                    acc_e, stream);
            });
          HIP_OK(ea);
          if (trace_partial)
            HIP_OK(launch_trace_gs(S.acc_slot, S.acc_entry, P.nnz, panel, P.panel_total, S.s, m, trace_nblk,
                                   trace_partial + int64_t(first) * trace_nblk, stream));
        };
        if (lfirst == hfirst + nhi) {
          sum_range(0, cnt, nhi > 0 ? hfirst : lfirst);  // contiguous in shift order
        } else {
          sum_range(0, nhi, hfirst);
          sum_range(nhi, cnt - nhi, lfirst);
        }
      }
    };
    // Does any pass run as several launch chains?  (the same test as in record)
    bool any_split = false;
    if (opt.split_streams > 0 && !prof && n_hi > 0 && n_hi < n) {
      const int npass = (n + nb - 1) / nb;
      const bool spread = npass > 1;
      int c0 = 0, h0 = 0;
      for (int b = 0; b < npass; ++b) {
        const int cnt = std::min(nb, n - c0);
        int nhi;
        if (spread) {
          const int h1 = static_cast<int>(int64_t(n_hi) * (c0 + cnt) / n);
          nhi = h1 - h0;
          h0 = h1;
        } else {
          nhi = std::max(0, std::min(cnt, n_hi - c0));
        }
        c0 += cnt;
        any_split = any_split || (nhi > 0 && nhi < cnt && P.flops_exec * cnt >= kSplitMinFlops);
      }
    }
    // Evaluations with several launch chains are not captured: device memory
    // that a graph with forked streams had run on stayed allocated after
    // hipFree on this runtime (measured: the whole workspace of every such
    // context), and their launches are long enough that graph replay gains
    // little there.
    if (!opt.use_graph || prof || any_split) {
      record();
      return;
    }
    // The whole evaluation (hundreds of launches) is captured once into a
    // hipGraph and replayed; anything that changes a launch argument (the
    // workspace, the shift arrays, the batch size, the precision split)
    // changes the key and triggers a new capture.
    std::vector<const void*> key = {ws, acc, status, alpha, w, S.m0, reinterpret_cast<const void*>(astride),
                                    reinterpret_cast<const void*>(static_cast<intptr_t>(S.tune_gen))};
    key.push_back(reinterpret_cast<const void*>(static_cast<intptr_t>(nb)));
    key.push_back(reinterpret_cast<const void*>(static_cast<intptr_t>(n)));
    key.push_back(reinterpret_cast<const void*>(static_cast<intptr_t>(n_hi)));
    key.push_back(reinterpret_cast<const void*>(static_cast<intptr_t>((add_m0 ? 1 : 0) | (spd_check ? 2 : 0) |
                                                                      (hcoef != 0.0 ? 4 : 0) | (edm ? 8 : 0))));
    if (trace_partial) {
      key.push_back(trace_partial);
      key.push_back(reinterpret_cast<const void*>(static_cast<intptr_t>(trace_nblk)));
    }
    if (edm) {
      int64_t kbits;
      static_assert(sizeof(kbits) == sizeof(S.kappa), "kappa bits");
      std::memcpy(&kbits, &S.kappa, sizeof(kbits));
      key.push_back(acc_e);
      key.push_back(S.d_cw);
      key.push_back(S.m1);
      key.push_back(reinterpret_cast<const void*>(static_cast<intptr_t>(kbits)));
    }
    if (!S.gexec || key != S.gkey) {
      if (S.gexec) HIP_OK(hipGraphExecDestroy(S.gexec));
      S.gexec = nullptr;
      if (opt.split_streams > 0) ensure_side(opt.split_streams);  // streams and events exist before the capture
      HIP_OK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
      try {
        record();
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      hipGraph_t g = nullptr;
      HIP_OK(hipStreamEndCapture(stream, &g));
      const hipError_t ie = hipGraphInstantiate(&S.gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIP_OK(ie);
      S.gkey = key;
    }
    HIP_OK(hipGraphLaunch(S.gexec, stream));
  }

  void read_status(int* st) {
    int w[4];
    HIP_OK(hipMemcpyAsync(w, status, 4 * sizeof(int), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    if (!recs.empty()) fold_profile();
    st[0] = w[0];
    st[1] = w[1];
  }

  // M0 = S^{-1} on the pattern: the real selected inversion of S (alpha = 1,
  // no H), which also tests S for positive definiteness through its pivots.
  void compute_m0(DevStruct& S) {
    const Plan& P = S.plan;
    std::vector<double2> one(1, make_double2(1.0, 0.0));
    std::vector<double> w1(1, 1.0);
    double2* da = upload(one, stream);
    double* dw = upload(w1, stream);
    if (!S.m0) {
      if (hipMalloc(&S.m0, P.nnz * sizeof(double)) != hipSuccess) fail(NDRHO_ENOMEM, "M0 allocation failed");
      S.allocs.push_back(S.m0);
    }
    try {
      evaluate(S, da, 0, dw, 1, 1, false, 0.0, 1);
      int st[2];
      read_status(st);
      if (st[0] || st[1]) fail(NDRHO_ENOTSPD, "S is not positive definite (a non-positive pivot of S)");
      HIP_OK(hipMemcpyAsync(S.m0, acc, P.nnz * sizeof(double), hipMemcpyDeviceToDevice, stream));
      HIP_OK(hipStreamSynchronize(stream));
    } catch (...) {
      (void)hipFree(da);
      (void)hipFree(dw);
      throw;
    }
    (void)hipFree(da);
    (void)hipFree(dw);
  }

  // M1 = S^{-1} H S^{-1} on the pattern, the first moment of G (G(Z) =
  // sum_k M_k Z^-(k+1), Eq. (12)).  From two shifts far up the imaginary
  // axis: Re G(iR) = -M1/R^2 + M3/R^4 - ..., so f(R) = -R^2 Re G(iR) = M1 -
  // M3/R^2 + ..., and (4 f(2R) - f(R))/3 = M1 + O(M5/R^4) (Richardson).
  // R = 1e3 max(1e-300, |H|_inf) balances that remainder, O((|S^-1 H|/R)^4),
  // against the rounding of Re G, O(u R |S^-1|) relative; both about 1e-12
  // for lattice Hamiltonians of a few eV.  FP64 for both shifts.
  void compute_m1(DevStruct& S) {
    const Plan& P = S.plan;
    if (!S.m1) {
      if (hipMalloc(&S.m1, P.nnz * sizeof(double)) != hipSuccess) fail(NDRHO_ENOMEM, "M1 allocation failed");
      S.allocs.push_back(S.m1);
    }
    if (S.h_inf == 0.0) {  // H = 0: M1 = 0
      HIP_OK(hipMemsetAsync(S.m1, 0, P.nnz * sizeof(double), stream));
      HIP_OK(hipStreamSynchronize(stream));
      S.m1_valid = true;
      return;
    }
    const double R = 1e3 * S.h_inf;
    std::vector<double2> a = {make_double2(0.0, R), make_double2(0.0, 2.0 * R)};
    std::vector<double> w = {R * R / 3.0, -16.0 * R * R / 3.0};
    double2* da = upload(a, stream);
    double* dw = upload(w, stream);
    try {
      evaluate(S, da, 0, dw, 2, 2, false, 1.0, 0);
      int st[2];
      read_status(st);
      if (st[0]) fail(NDRHO_ESINGULAR, "a tiny pivot occurred in i R S - H (first moment of G)");
      HIP_OK(hipMemcpyAsync(S.m1, acc, P.nnz * sizeof(double), hipMemcpyDeviceToDevice, stream));
      HIP_OK(hipStreamSynchronize(stream));
    } catch (...) {
      (void)hipFree(da);
      (void)hipFree(dw);
      throw;
    }
    (void)hipFree(da);
    (void)hipFree(dw);
    S.m1_valid = true;
  }

  // rho of the structure's current poles (CSR order, host) and the deviation
  // of its electron count Tr(rho S) = sum_ij rho_ij S_ji (Eq. (40)) from n_ideal.
  double delta_n(DevStruct& S, double n_ideal, std::vector<double>& rho) {
    const Plan& P = S.plan;
    evaluate(S, S.d_alpha, 0, S.d_w, S.n_shifts, S.n_hi, S.add_m0, 1.0, 0);
    HIP_OK(launch_scatter(S.acc_entry, P.nnz, acc, outbuf, stream));
    int st[2];
    read_status(st);
    if (st[0]) fail(NDRHO_ESINGULAR, "a zero, tiny or non-finite pivot occurred in alpha S - H");
    rho.resize(P.nnz);
    HIP_OK(hipMemcpyAsync(rho.data(), outbuf, P.nnz * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    double tr = 0.0;
    for (int64_t e = 0; e < P.nnz; ++e) tr += rho[e] * S.s_host[e];  // S symmetric: S_ji = S_ij
    return tr - n_ideal;
  }

  // Tr(G(alpha_k) S) for n shifts (FP64 front updates for all of them).
  std::vector<double2> green_traces(DevStruct& S, const std::vector<double2>& alpha) {
    const Plan& P = S.plan;
    const int n = static_cast<int>(alpha.size());
    const int nblk = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(64, (P.nnz + 255) / 256)));
    std::vector<double> w(n, 0.0);
    double2* da = upload(alpha, stream);
    double* dw = upload(w, stream);
    double2* part = nullptr;
    std::vector<double2> hp(static_cast<size_t>(n) * nblk);
    try {
      if (hipMalloc(&part, hp.size() * sizeof(double2)) != hipSuccess) fail(NDRHO_ENOMEM, "trace buffer");
      evaluate(S, da, 0, dw, n, n, false, 1.0, 0, false, part, nblk);
      int st[2];
      read_status(st);
      if (st[0]) fail(NDRHO_ESINGULAR, "a zero, tiny or non-finite pivot occurred in alpha S - H");
      HIP_OK(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double2), hipMemcpyDeviceToHost, stream));
      HIP_OK(hipStreamSynchronize(stream));
    } catch (...) {
      (void)hipFree(da);
      (void)hipFree(dw);
      if (part) (void)hipFree(part);
      throw;
    }
    (void)hipFree(da);
    (void)hipFree(dw);
    (void)hipFree(part);
    // the graph captured for these buffers must not be replayed after they are freed
    if (S.gexec) (void)hipGraphExecDestroy(S.gexec);
    S.gexec = nullptr;
    S.gkey.clear();
    std::vector<double2> tr(n, make_double2(0.0, 0.0));
    for (int k = 0; k < n; ++k)
      for (int b = 0; b < nblk; ++b) {
        tr[k].x += hp[static_cast<size_t>(k) * nblk + b].x;
        tr[k].y += hp[static_cast<size_t>(k) * nblk + b].y;
      }
    return tr;
  }

  // Energy density matrix buffers of nnz entries.
  void ensure_edm(int64_t nnz) {
    if (nnz <= acc_e_len) return;
    if (acc_e) HIP_OK(hipFree(acc_e));
    if (outbuf_e) HIP_OK(hipFree(outbuf_e));
    acc_e = outbuf_e = nullptr;
    acc_e_len = 0;
    if (hipMalloc(&acc_e, nnz * sizeof(double)) != hipSuccess || hipMalloc(&outbuf_e, nnz * sizeof(double)) != hipSuccess)
      fail(NDRHO_ENOMEM, "energy density matrix buffers");
    acc_e_len = nnz;
  }

  // Joined plan for a list of structures (built, uploaded and given its own
  // M0 on first use; values are copied from the member structures).
  DevStruct& get_union(const std::vector<int32_t>& ids) {
    auto it = unions.find(ids);
    if (it != unions.end()) return *it->second;
    std::vector<const Plan*> parts;
    for (int32_t id : ids) parts.push_back(&get(id).plan);
    std::unique_ptr<DevStruct> ds(new DevStruct());
    try {
      join_plans(ds->plan, parts);
      const Plan& P = ds->plan;
      for (double** dst : {&ds->h, &ds->s}) {
        if (hipMalloc(dst, P.nnz * sizeof(double)) != hipSuccess) fail(NDRHO_ENOMEM, "batch allocation failed");
        ds->allocs.push_back(*dst);
      }
      for (size_t k = 0; k < ids.size(); ++k) {
        const DevStruct& m = get(ids[k]);
        const size_t bytes = m.plan.nnz * sizeof(double);
        HIP_OK(hipMemcpyAsync(ds->h + P.struct_nnz_off[k], m.h, bytes, hipMemcpyDeviceToDevice, stream));
        HIP_OK(hipMemcpyAsync(ds->s + P.struct_nnz_off[k], m.s, bytes, hipMemcpyDeviceToDevice, stream));
      }
      upload_plan(*ds, stream, opt.precision);
      // structure of every sorted slot (energy weights differ per structure)
      std::vector<int32_t> sid(P.nnz);
      for (int64_t k = 0; k < P.nnz; ++k)
        sid[k] = static_cast<int32_t>(std::upper_bound(P.struct_nnz_off.begin(), P.struct_nnz_off.end(),
                                                       static_cast<int64_t>(P.acc_entry[k])) -
                                      P.struct_nnz_off.begin()) - 1;
      ds->acc_sid = ds->put(sid, stream);
      for (int32_t id : ids) ds->h_inf = std::max(ds->h_inf, get(id).h_inf);
      HIP_OK(hipStreamSynchronize(stream));
      compute_m0(*ds);
    } catch (...) {
      ds->release();
      throw;
    }
    DevStruct& ref = *ds;
    unions[ids] = std::move(ds);
    return ref;
  }

  // Validate a batch, get its joined plan and fill its shift table
  // (per-structure alpha side by side with stride n_shifts, common weights).
  DevStruct& prepare_batch(const std::vector<int32_t>& ids) {
    const int32_t k = static_cast<int32_t>(ids.size());
    {
      std::vector<int32_t> sorted = ids;
      std::sort(sorted.begin(), sorted.end());
      if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        fail(NDRHO_EINVAL, "a structure appears twice in the batch");
    }
    const DevStruct& first = get(ids[0]);
    for (int32_t id : ids) {
      const DevStruct& m = get(id);
      if (m.n_shifts < 1) fail(NDRHO_ESTATE, "set_poles (or set_shifts) has not been called for a batch member");
      if (m.n_shifts != first.n_shifts || m.w_host != first.w_host || m.add_m0 != first.add_m0 ||
          m.n_hi != first.n_hi)
        fail(NDRHO_EINVAL, "batch members need the same number of poles, weights (beta) and M0 flag");
    }
    DevStruct& U = get_union(ids);
    const int n = first.n_shifts;
    if (U.n_shifts != n || !U.d_alpha) {
      if (U.d_alpha) HIP_OK(hipFree(U.d_alpha));
      if (U.d_w) HIP_OK(hipFree(U.d_w));
      if (U.d_cw) HIP_OK(hipFree(U.d_cw));
      U.d_alpha = nullptr;
      U.d_w = nullptr;
      U.d_cw = nullptr;
      if (hipMalloc(&U.d_alpha, sizeof(double2) * n * k) != hipSuccess ||
          hipMalloc(&U.d_w, sizeof(double) * n) != hipSuccess ||
          hipMalloc(&U.d_cw, sizeof(double2) * n * k) != hipSuccess)
        fail(NDRHO_ENOMEM, "batch shift allocation failed");
      U.n_shifts = n;
    }
    U.cf_poles = true;
    for (int32_t i = 0; i < k; ++i) {
      const DevStruct& m = get(ids[i]);
      HIP_OK(hipMemcpyAsync(U.d_alpha + int64_t(i) * n, m.d_alpha, sizeof(double2) * n, hipMemcpyDeviceToDevice,
                            stream));
      HIP_OK(hipMemcpyAsync(U.d_cw + int64_t(i) * n, m.d_cw, sizeof(double2) * n, hipMemcpyDeviceToDevice, stream));
      U.cf_poles = U.cf_poles && m.cf_poles;
    }
    HIP_OK(hipMemcpyAsync(U.d_w, first.d_w, sizeof(double) * n, hipMemcpyDeviceToDevice, stream));
    U.n_hi = first.n_hi;
    U.add_m0 = first.add_m0;
    U.kappa = first.kappa;  // the members share their weights
    return U;
  }

  void drop_unions() {
    for (auto& u : unions) u.second->release();
    unions.clear();
  }

  // Tables of the solve X^{-1} y through the stored factor (Appendix B):
  // fronts by depth, the children's inverse maps, update-row lists, and the
  // tiles of the forward gather and of the grouped products of each step.
  void build_eigen_plan(DevStruct& S) {
    DevStruct::EigenPlan& E = S.eig;
    if (E.built) return;
    const Plan& P = S.plan;
    const int nf = static_cast<int>(P.fronts.size());
    std::vector<int> order(nf), pos(nf);
    for (int f = 0; f < nf; ++f) order[f] = f;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return P.fronts[a].depth < P.fronts[b].depth; });
    for (int i = 0; i < nf; ++i) pos[order[i]] = i;
    std::vector<int64_t> wrow(nf, 0), urow(nf, 0);
    int64_t wr = 0, ur = 0;
    std::vector<int32_t> urows;
    for (int f = 0; f < nf; ++f) {
      wrow[f] = wr;
      wr += P.fronts[f].nu;
      urow[f] = ur;
      ur += P.fronts[f].nu;
      urows.insert(urows.end(), P.fronts[f].u.begin(), P.fronts[f].u.end());
    }
    E.w_rows = std::max<int64_t>(wr, 1);
    if (urows.empty()) urows.push_back(0);
    std::vector<SolveFront> fr(nf);
    std::vector<SolveChild> kids;
    std::vector<int32_t> inv;
    for (int i = 0; i < nf; ++i) {
      const Front& F = P.fronts[order[i]];
      SolveFront d{F.j0, wrow[order[i]] * EIG_NR, F.nj, F.nu, static_cast<int32_t>(kids.size()),
                   static_cast<int32_t>(F.children.size())};
      for (int c : F.children) {
        const Front& C = P.fronts[c];
        kids.push_back(SolveChild{wrow[c] * EIG_NR, static_cast<int64_t>(inv.size()), C.nu, 0});
        std::vector<int32_t> m(F.nj + F.nu, -1);
        for (int k = 0; k < C.nu; ++k) m[C.rel[k]] = k;
        inv.insert(inv.end(), m.begin(), m.end());
      }
      fr[i] = d;
    }
    if (kids.empty()) kids.push_back(SolveChild{0, 0, 0, 0});
    if (inv.empty()) inv.push_back(-1);
    const int nd = P.n_levels;
    std::vector<SolveTile> gt;
    std::vector<TsProb> probs;
    std::vector<TsTile> tt;
    auto add_prob = [&](const TsProb& p) {
      const int32_t id = static_cast<int32_t>(probs.size());
      probs.push_back(p);
      for (int m0 = 0; m0 < p.m; m0 += 64) tt.push_back(TsTile{id, m0});
    };
    E.g_begin.assign(nd + 1, 0);
    E.f_begin.assign(nd + 1, 0);
    E.b_begin.assign(nd + 1, 0);
    auto range_of = [&](int d, int& lo, int& hi) {
      lo = static_cast<int>(std::lower_bound(order.begin(), order.end(), d,
                                             [&](int f, int v) { return P.fronts[f].depth < v; }) - order.begin());
      hi = static_cast<int>(std::upper_bound(order.begin(), order.end(), d,
                                             [&](int v, int f) { return v < P.fronts[f].depth; }) - order.begin());
    };
    for (int d = 0; d < nd; ++d) {  // forward gather tiles and forward products, per depth
      int lo, hi;
      range_of(d, lo, hi);
      E.g_begin[d] = static_cast<int64_t>(gt.size());
      for (int i = lo; i < hi; ++i)
        for (int r0 = 0; r0 < fr[i].nj + fr[i].nu; r0 += EIG_GROWS) gt.push_back(SolveTile{i, r0});
      E.f_begin[d] = static_cast<int64_t>(tt.size());
      for (int i = lo; i < hi; ++i) {
        const Front& F = P.fronts[order[i]];
        if (F.nu == 0) continue;
        add_prob(TsProb{F.l_off, F.j0, wrow[order[i]], wrow[order[i]], F.nu, F.nu, F.nj, 0});
      }
    }
    E.g_begin[nd] = static_cast<int64_t>(gt.size());
    E.f_begin[nd] = static_cast<int64_t>(tt.size());
    E.d_begin = static_cast<int64_t>(tt.size());
    for (int i = 0; i < nf; ++i) {  // diagonal: every front at once
      const Front& F = P.fronts[order[i]];
      add_prob(TsProb{F.panel_off, F.j0, F.j0, 0, F.nj + F.nu, F.nj, F.nj, 0});
    }
    E.d_count = static_cast<int64_t>(tt.size()) - E.d_begin;
    for (int d = 0; d < nd; ++d) {  // backward products, per depth
      int lo, hi;
      range_of(d, lo, hi);
      E.b_begin[d] = static_cast<int64_t>(tt.size());
      for (int i = lo; i < hi; ++i) {
        const Front& F = P.fronts[order[i]];
        add_prob(TsProb{F.l_off, urow[order[i]], F.j0, F.j0, std::max(F.nu, 1), F.nj, F.nu, 0});
      }
    }
    E.b_begin[nd] = static_cast<int64_t>(tt.size());
    E.fronts = S.put(fr, stream);
    E.kids = S.put(kids, stream);
    E.inv = S.put(inv, stream);
    E.urows = S.put(urows, stream);
    E.gtiles = S.put(gt, stream);
    E.probs = S.put(probs, stream);
    E.ttiles = S.put(tt, stream);
    E.perm = S.put(P.perm, stream);
    E.iperm = S.put(P.iperm, stream);
    E.rp = S.put(P.row_ptr, stream);
    E.col = S.put(P.col, stream);
    HIP_OK(hipStreamSynchronize(stream));
    E.built = true;
  }

  // x = X^{-1} y through the factor held in the workspace (pole 0): the
  // three steps of Eqs. (B8)-(B14); y, z, z2, x: n x EIG_NR complex in the
  // permuted order; w: the update blocks.
  void solve_factor(DevStruct& S, const double2* y, double2* z, double2* z2, double2* x, double2* w) {
    const Plan& P = S.plan;
    const DevStruct::EigenPlan& E = S.eig;
    double2* bufs[BUF_COUNT];
    int64_t strides[BUF_COUNT];
    layout(P, 1, bufs, strides);
    const double2* L = bufs[BUF_L];
    const double2* panel = bufs[BUF_PANEL];
    for (int d = P.n_levels - 1; d >= 0; --d) {
      HIP_OK(launch_solve_gather(E.fronts, E.kids, E.inv, E.gtiles + E.g_begin[d], E.g_begin[d + 1] - E.g_begin[d],
                                 y, z, w, stream));
      HIP_OK(launch_tsgemm(TS_FORWARD, E.probs, E.ttiles + E.f_begin[d], E.f_begin[d + 1] - E.f_begin[d], L, z,
                           nullptr, w, w, stream));
    }
    HIP_OK(launch_tsgemm(TS_DIAGONAL, E.probs, E.ttiles + E.d_begin, E.d_count, panel, z, nullptr, nullptr, z2,
                         stream));
    for (int d = 0; d < P.n_levels; ++d)
      HIP_OK(launch_tsgemm(TS_BACKWARD, E.probs, E.ttiles + E.b_begin[d], E.b_begin[d + 1] - E.b_begin[d], L, x,
                           E.urows, z2, x, stream));
  }

  void set_shifts(DevStruct& S, const std::vector<double2>& alpha_in, const std::vector<double>& w_in,
                  bool add_m0, bool cf) {
    // Mixed mode keeps in FP64 the fp64_poles shifts nearest the real axis,
    // the fp64_far_poles farthest from it, and any with |Im alpha| below
    // fp64_pole_im.  Those are moved to the front (stable order otherwise):
    // the pole sum is still taken in one fixed order.
    const int n = static_cast<int>(alpha_in.size());
    std::vector<double2> alpha = alpha_in;
    std::vector<double> w = w_in;
    int hi = n;
    if (opt.precision != NDRHO_FP64) {
      std::vector<int> by_im(n);
      for (int i = 0; i < n; ++i) by_im[i] = i;
      std::stable_sort(by_im.begin(), by_im.end(),
                       [&](int a, int b) { return std::fabs(alpha_in[a].y) < std::fabs(alpha_in[b].y); });
      std::vector<char> keep(n, 0);
      for (int r = 0; r < n; ++r) {
        const int i = by_im[r];
        if (r < opt.fp64_poles || r >= n - opt.fp64_far_poles || std::fabs(alpha_in[i].y) < opt.fp64_pole_im)
          keep[i] = 1;
      }
      alpha.clear();
      w.clear();
      for (int pass = 1; pass >= 0; --pass)
        for (int i = 0; i < n; ++i)
          if (keep[i] == pass) {
            alpha.push_back(alpha_in[i]);
            w.push_back(w_in[i]);
          }
      hi = 0;
      for (int i = 0; i < n; ++i) hi += keep[i];
    }
    S.n_hi = hi;
    // weights of the energy density matrix, c_p = w_p alpha_p, and
    // kappa = (4/beta) sum_p R_p = -sum_p w_p (Eqs. (10), (11))
    std::vector<double2> cw(alpha.size());
    double kappa = 0.0;
    for (size_t p = 0; p < alpha.size(); ++p) {
      cw[p] = make_double2(w[p] * alpha[p].x, w[p] * alpha[p].y);
      kappa -= w[p];
    }
    if (S.d_alpha) HIP_OK(hipFree(S.d_alpha));
    if (S.d_w) HIP_OK(hipFree(S.d_w));
    if (S.d_cw) HIP_OK(hipFree(S.d_cw));
    S.d_alpha = nullptr;
    S.d_w = nullptr;
    S.d_cw = nullptr;
    S.d_alpha = upload(alpha, stream);
    S.d_w = upload(w, stream);
    S.d_cw = upload(cw, stream);
    HIP_OK(hipStreamSynchronize(stream));
    S.n_shifts = static_cast<int>(alpha.size());
    S.add_m0 = add_m0;
    S.cf_poles = cf;
    S.kappa = kappa;
    S.w_host = w;
  }
};

namespace {

template <class F>
int guarded(ndrho_ctx* ctx, F&& f) {
  try {
    f();
    return NDRHO_OK;
  } catch (const Error& e) {
    if (ctx) ctx->err = e.what();
    else g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->err = "host allocation failed";
    else g_err = "host allocation failed";
    return NDRHO_ENOMEM;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    else g_err = e.what();
    return NDRHO_EINVAL;
  }
}

}  // namespace

struct ndrho_plan {
  Plan plan;
};

extern "C" {

int ndrho_default_options(ndrho_options* opt) {
  if (!opt) return NDRHO_EINVAL;
  opt->leaf_rows = 32;
  opt->precision = NDRHO_FP64;
  opt->pole_batch = 0;
  opt->mem_fraction = 0.8;
  opt->verbose = 0;
  opt->fp64_poles = 12;
  opt->fp64_pole_im = 0.05;
  opt->fp64_far_poles = 12;
  opt->use_graph = 1;
  opt->gemm_variant = -1;
  opt->fp64_small_tiles = -1;
  opt->split_streams = 0;
  opt->long_tail = 0.0;
  opt->small_fronts = 0;
  opt->pivot_variant = 0;
  return NDRHO_OK;
}

int ndrho_create(ndrho_ctx** out, int device, void* hip_stream, const ndrho_options* opt) {
  if (!out) {
    g_err = "out is NULL";
    return NDRHO_EINVAL;
  }
  *out = nullptr;
  std::unique_ptr<ndrho_ctx> c(new (std::nothrow) ndrho_ctx());
  if (!c) return NDRHO_ENOMEM;
  int rc = guarded(nullptr, [&] {
    ndrho_default_options(&c->opt);
    if (opt) c->opt = *opt;
    if (c->opt.leaf_rows < 1) fail(NDRHO_EINVAL, "leaf_rows must be >= 1");
    if (c->opt.precision != NDRHO_FP64 && c->opt.precision != NDRHO_MIXED_FP32 &&
        c->opt.precision != NDRHO_MIXED_BF16X3)
      fail(NDRHO_EUNSUPPORTED, "precision must be NDRHO_FP64, NDRHO_MIXED_FP32 or NDRHO_MIXED_BF16X3");
    if (c->opt.fp64_poles < 0 || c->opt.fp64_far_poles < 0 || !(c->opt.fp64_pole_im >= 0.0))
      fail(NDRHO_EINVAL, "invalid FP64 pole rule");
    if (c->opt.fp64_small_tiles < -1 || c->opt.fp64_small_tiles > 1) fail(NDRHO_EINVAL, "invalid fp64_small_tiles");
    if (!(c->opt.long_tail == 0.0 || c->opt.long_tail >= 1.0)) fail(NDRHO_EINVAL, "long_tail must be 0 or >= 1");
    if (c->opt.small_fronts != 0 && c->opt.small_fronts != 1) fail(NDRHO_EINVAL, "small_fronts must be 0 or 1");
    if (c->opt.split_streams < 0 || c->opt.split_streams > ndrho_ctx::kMaxChains)
      fail(NDRHO_EINVAL, "invalid split_streams");
    if (c->opt.pivot_variant < -1 || c->opt.pivot_variant >= V_COUNT ||
        (c->opt.pivot_variant >= 0 && !variant_allowed(c->opt.precision, c->opt.pivot_variant)))
      fail(NDRHO_EINVAL, "invalid pivot_variant for this precision");
    if (c->opt.gemm_variant < -1 || c->opt.gemm_variant >= V_COUNT ||
        (c->opt.gemm_variant >= 0 && !variant_allowed(c->opt.precision, c->opt.gemm_variant)))
      fail(NDRHO_EINVAL, "invalid gemm_variant for this precision");
    if (c->opt.pole_batch < 0) fail(NDRHO_EINVAL, "pole_batch must be >= 0");
    if (!(c->opt.mem_fraction > 0.0 && c->opt.mem_fraction <= 1.0)) fail(NDRHO_EINVAL, "mem_fraction must be in (0, 1]");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) fail(NDRHO_EDEVICE, "no HIP device available");
    if (device < 0 || device >= count) fail(NDRHO_EDEVICE, "device index out of range");
    HIP_OK(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      fail(NDRHO_EDEVICE, std::string("this library is built for gfx950, device is ") + prop.gcnArchName);
    c->device = device;
    if (hip_stream) {
      c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      HIP_OK(hipStreamCreate(&c->stream));
      c->own_stream = true;
    }
    if (hipMalloc(&c->status, 4 * sizeof(int)) != hipSuccess) fail(NDRHO_ENOMEM, "status allocation failed");
    c->scratch = scratch_addr(device);
  });
  if (rc == NDRHO_OK) *out = c.release();
  return rc;
}

int ndrho_destroy(ndrho_ctx* ctx) {
  if (!ctx) return NDRHO_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
  return NDRHO_OK;
}

const char* ndrho_last_error(const ndrho_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

namespace {

int set_structure(ndrho_ctx* ctx, int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* H,
                  const double* S, const double* coords, const double* cell, int32_t* struct_id) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    if (!H || !S || !struct_id) fail(NDRHO_EINVAL, "H, S and struct_id are required");
    if (cell && !coords) fail(NDRHO_EINVAL, "a periodic cell needs the coordinates");
    HIP_OK(hipSetDevice(ctx->device));
    validate_csr(n, row_ptr, col_idx, H, S);
    if (coords)
      for (int64_t i = 0; i < 3 * n; ++i)
        if (!std::isfinite(coords[i])) fail(NDRHO_EINVAL, "non-finite coordinate");
    std::unique_ptr<DevStruct> ds(new DevStruct());
    try {
      build_plan(ds->plan, n, row_ptr, col_idx, coords, ctx->opt.leaf_rows, ctx->opt.long_tail, cell,
                 ctx->opt.small_fronts != 0);
      Plan& P = ds->plan;
      hipStream_t st = ctx->stream;
      std::vector<double> hv(H, H + P.nnz), sv(S, S + P.nnz);
      ds->h = ds->put(hv, st);
      ds->s = ds->put(sv, st);
      ds->h_inf = row_sum_norm(P, H);
      ds->s_host = sv;
      ds->h_host = hv;
      upload_plan(*ds, st, ctx->opt.precision);
      HIP_OK(hipStreamSynchronize(st));
      ctx->compute_m0(*ds);
    } catch (...) {
      ds->release();
      throw;
    }
    ctx->structs.push_back(std::move(ds));
    *struct_id = static_cast<int32_t>(ctx->structs.size()) - 1;
  });
}

}  // namespace

int ndrho_set_structure(ndrho_ctx* ctx, int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* H,
                        const double* S, const double* coords, int32_t* struct_id) {
  return set_structure(ctx, n, row_ptr, col_idx, H, S, coords, nullptr, struct_id);
}

int ndrho_set_structure_periodic(ndrho_ctx* ctx, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                                 const double* H, const double* S, const double* coords, const double* cell,
                                 int32_t* struct_id) {
  if (!cell) {
    if (ctx) ctx->err = "cell is required";
    return NDRHO_EINVAL;
  }
  return set_structure(ctx, n, row_ptr, col_idx, H, S, coords, cell, struct_id);
}

int ndrho_update_values(ndrho_ctx* ctx, int32_t struct_id, const double* H, const double* S) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    DevStruct& ds = ctx->get(struct_id);
    if (!H || !S) fail(NDRHO_EINVAL, "H and S are required");
    const Plan& P = ds.plan;
    validate_csr(P.n, P.row_ptr.data(), P.col.data(), H, S);
    HIP_OK(hipSetDevice(ctx->device));
    HIP_OK(hipMemcpyAsync(ds.h, H, P.nnz * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIP_OK(hipMemcpyAsync(ds.s, S, P.nnz * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    ds.h_inf = row_sum_norm(P, H);
    ds.m1_valid = false;
    ds.s_host.assign(S, S + P.nnz);
    ds.h_host.assign(H, H + P.nnz);
    ctx->drop_unions();
    ctx->compute_m0(ds);
  });
}

namespace {

// Shifts and weights of Eq. (8) for the continued-fraction poles at mu.
void set_cf_poles(ndrho_ctx* ctx, DevStruct& ds, double mu, double beta, int32_t n_poles) {
  if (n_poles < 1 || n_poles > 100000) fail(NDRHO_EINVAL, "n_poles must be in [1, 100000]");
  if (!(beta > 0.0) || !std::isfinite(beta)) fail(NDRHO_EINVAL, "beta must be positive and finite");
  if (!std::isfinite(mu)) fail(NDRHO_EINVAL, "mu must be finite");
  std::vector<double> z(n_poles), r(n_poles), w(n_poles);
  cf_poles(n_poles, z.data(), r.data());
  std::vector<double2> a(n_poles);
  for (int p = 0; p < n_poles; ++p) {
    a[p] = make_double2(mu, z[p] / beta);  // alpha_p = mu + i z_p / beta
    w[p] = -(4.0 / beta) * r[p];          // Im(-(4i/beta) G R) = -(4/beta) R Re G
  }
  ctx->set_shifts(ds, a, w, true, true);
}

// Trial mu from three (mu, dN) points by the quadratic through them (Muller,
// Eqs. (45)-(46)), in coordinates x = mu - mu[0]; the root taken is the one
// where dN rises through zero (gradient 2 a x + b > 0), in the form without
// cancellation for either sign of b.  NaN when the quadratic has no such root.
double muller_step(const double* mu, const double* dn) {
  const double x1 = mu[1] - mu[0], x2 = mu[2] - mu[0];
  const double d1 = (dn[1] - dn[0]) / x1, d2 = (dn[2] - dn[0]) / x2;
  const double a = (d2 - d1) / (x2 - x1);
  const double b = d1 - a * x1;
  const double c = dn[0];
  const double disc = b * b - 4.0 * a * c;
  if (!(disc >= 0.0)) return std::nan("");
  const double sq = std::sqrt(disc);
  double x;
  if (b >= 0.0) {
    x = (b + sq) != 0.0 ? -2.0 * c / (b + sq) : std::nan("");
  } else {
    x = a != 0.0 ? (-b + sq) / (2.0 * a) : std::nan("");
  }
  return mu[0] + x;
}

// Eigenpairs of a real symmetric n x n matrix a (row-major) by cyclic Jacobi
// rotations: eigenvalues w ascending, eigenvectors as the columns of v
// (row-major n x n).
void sym_eig(int n, std::vector<double> a, std::vector<double>& w, std::vector<double>& v) {
  v.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) v[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += a[i * n + j] * a[i * n + j];
        if (i != j) off += a[i * n + j] * a[i * n + j];
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[p * n + q];
        if (apq == 0.0) continue;
        const double th = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - sn * akq;
          a[k * n + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - sn * aqk;
          a[q * n + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = v[k * n + p], vkq = v[k * n + q];
          v[k * n + p] = c * vkp - sn * vkq;
          v[k * n + q] = sn * vkp + c * vkq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a[x * n + x] < a[y * n + y]; });
  std::vector<double> vs(static_cast<size_t>(n) * n);
  w.resize(n);
  for (int j = 0; j < n; ++j) {
    w[j] = a[idx[j] * n + idx[j]];
    for (int k = 0; k < n; ++k) vs[k * n + j] = v[k * n + idx[j]];
  }
  v.swap(vs);
}

// Counter-based uniform numbers in [-1, 1) (SplitMix64 of the counter).
double splitmix_uniform(uint64_t i) {
  uint64_t z = i + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return static_cast<double>(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

}  // namespace

int ndrho_set_poles(ndrho_ctx* ctx, int32_t struct_id, double mu, double beta, int32_t n_poles) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    DevStruct& ds = ctx->get(struct_id);
    HIP_OK(hipSetDevice(ctx->device));
    set_cf_poles(ctx, ds, mu, beta, n_poles);
  });
}

int ndrho_green_traces(ndrho_ctx* ctx, int32_t struct_id, int32_t n, const double* alpha_re, const double* alpha_im,
                       double* tr_re, double* tr_im) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    DevStruct& ds = ctx->get(struct_id);
    if (n < 1 || !alpha_re || !alpha_im || !tr_re || !tr_im) fail(NDRHO_EINVAL, "n >= 1 and all arrays are required");
    std::vector<double2> a(n);
    for (int k = 0; k < n; ++k) {
      if (!std::isfinite(alpha_re[k]) || !std::isfinite(alpha_im[k])) fail(NDRHO_EINVAL, "non-finite shift");
      a[k] = make_double2(alpha_re[k], alpha_im[k]);
    }
    HIP_OK(hipSetDevice(ctx->device));
    const std::vector<double2> tr = ctx->green_traces(ds, a);
    for (int k = 0; k < n; ++k) tr_re[k] = tr[k].x, tr_im[k] = tr[k].y;
  });
}

namespace {

// Step (2) of the mu search (Eqs. (41)-(43)): the change of the electron
// count when mu moves from mu_i to mu_t is estimated as
//   dN(mu_t) = int dE drho(E) [f((E - mu_t)/kT) - f((E - mu_i)/kT)],
//   drho(E) = -(2/pi) Im Tr(G(E + i eta) S),   eta = 0.01 eV,
// by the trapezoidal rule on n_grid points over [mu_i - L, mu_i + L], and mu_t
// solves dN_i + dN(mu_t) = 0 by bisection inside the window (the estimate is
// monotone in mu_t since drho >= 0).
double retarded_estimate(ndrho_ctx* ctx, DevStruct& ds, double mu_i, double dn_i, double beta, int n_grid,
                         double half_width) {
  const double eta = 0.01;
  std::vector<double2> a(n_grid);
  const double h = 2.0 * half_width / (n_grid - 1);
  for (int k = 0; k < n_grid; ++k) a[k] = make_double2(mu_i - half_width + h * k, eta);
  const std::vector<double2> tr = ctx->green_traces(ds, a);
  std::vector<double> drho(n_grid);
  for (int k = 0; k < n_grid; ++k) drho[k] = -(2.0 / M_PI) * tr[k].y;
  auto fermi = [&](double x) { return x > 0 ? std::exp(-x) / (1.0 + std::exp(-x)) : 1.0 / (1.0 + std::exp(x)); };
  auto dn_of = [&](double mu_t) {
    double acc = 0.0;
    for (int k = 0; k < n_grid; ++k) {
      const double e = a[k].x;
      const double df = fermi(beta * (e - mu_t)) - fermi(beta * (e - mu_i));
      acc += (k == 0 || k == n_grid - 1 ? 0.5 : 1.0) * h * drho[k] * df;
    }
    return acc;
  };
  double lo = mu_i - half_width, hi = mu_i + half_width;
  for (int it = 0; it < 200 && hi - lo > 1e-12 * std::max(1.0, std::fabs(mu_i)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (dn_i + dn_of(mid) < 0.0) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

int ndrho_find_mu(ndrho_ctx* ctx, int32_t struct_id, double n_ideal, double beta, int32_t n_poles, double mu0,
                  double tol, int32_t max_iter, int32_t retarded_step, double* mu_out, double* delta_n_out,
                  int32_t* iters_out, double* rho_out) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    DevStruct& ds = ctx->get(struct_id);
    const Plan& P = ds.plan;
    if (!mu_out) fail(NDRHO_EINVAL, "mu_out is required");
    if (!(n_ideal > 0.0 && n_ideal < 2.0 * static_cast<double>(P.n)))
      fail(NDRHO_EINVAL, "n_ideal must lie strictly between 0 and 2 n");
    if (!(tol > 0.0) || max_iter < 1) fail(NDRHO_EINVAL, "tol > 0 and max_iter >= 1 are required");
    HIP_OK(hipSetDevice(ctx->device));
    std::vector<double> rho;
    std::vector<double> hm, hd;  // history of (mu, dN)
    auto eval = [&](double mu) {
      set_cf_poles(ctx, ds, mu, beta, n_poles);
      const double d = ctx->delta_n(ds, n_ideal, rho);
      hm.push_back(mu);
      hd.push_back(d);
      return d;
    };
    // bracket: dN(lo) < 0 < dN(hi) (the count rises with mu)
    double lo = -HUGE_VAL, hi = HUGE_VAL;
    auto bracket = [&](double mu, double d) {
      if (d < 0.0 && mu > lo) lo = mu;
      if (d > 0.0 && mu < hi) hi = mu;
    };
    double mu = mu0, d = eval(mu0);
    bracket(mu, d);
    double step = 10.0 / beta;  // first move: ten kT against the sign of dN
    if (retarded_step && std::fabs(d) > 1.0 && std::fabs(d) > tol && max_iter > 1) {
      // far from the count: one estimate from the retarded Green function
      // (step (2)) on 2 n_poles points over mu0 +- max(2 eV, 40 kT)
      const double half = std::max(2.0, 40.0 / beta);
      const double t = retarded_estimate(ctx, ds, mu, d, beta, 2 * n_poles, half);
      step = std::max(std::fabs(t - mu), 1e-3 / beta) * 2.0;
      mu = t;
      d = eval(mu);
      bracket(mu, d);
    }
    while (std::fabs(d) > tol && static_cast<int32_t>(hm.size()) < max_iter) {
      double t = std::nan("");
      const size_t k = hm.size();
      if (k >= 3) {
        // three points with the smallest |dN|, both signs among them when
        // the history has both (interpolation rather than extrapolation)
        std::vector<size_t> idx(k);
        for (size_t i = 0; i < k; ++i) idx[i] = i;
        std::sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return std::fabs(hd[a]) < std::fabs(hd[b]); });
        std::vector<size_t> pick(idx.begin(), idx.begin() + 3);
        const bool mixed = (hd[pick[0]] < 0) != (hd[pick[1]] < 0) || (hd[pick[0]] < 0) != (hd[pick[2]] < 0);
        if (!mixed)
          for (size_t i = 3; i < k; ++i)
            if ((hd[idx[i]] < 0) != (hd[pick[0]] < 0)) {
              pick[2] = idx[i];
              break;
            }
        const double m3[3] = {hm[pick[0]], hm[pick[1]], hm[pick[2]]};
        const double d3[3] = {hd[pick[0]], hd[pick[1]], hd[pick[2]]};
        if (m3[0] != m3[1] && m3[0] != m3[2] && m3[1] != m3[2]) t = muller_step(m3, d3);
      }
      if (!std::isfinite(t) && k >= 2) {
        // line through the last two points (Eq. (44), with the denominator
        // dN_i - dN_j: the printed mu_i - mu_j does not give the zero)
        const double mi = hm[k - 1], di = hd[k - 1], mj = hm[k - 2], dj = hd[k - 2];
        if (di != dj) t = (mj * di - mi * dj) / (di - dj);
      }
      if (!std::isfinite(t)) t = mu - (d > 0.0 ? step : -step);
      // safeguards: stay strictly inside a known bracket (else bisect);
      // with a one-sided bracket move at least as far as the last step
      if (std::isfinite(lo) && std::isfinite(hi)) {
        if (!(t > lo && t < hi)) t = 0.5 * (lo + hi);
      } else if (std::isfinite(lo) && !(t > lo)) {
        t = lo + 2.0 * step;
      } else if (std::isfinite(hi) && !(t < hi)) {
        t = hi - 2.0 * step;
      }
      step = std::max(std::fabs(t - mu), 1e-3 / beta) * 2.0;
      mu = t;
      d = eval(mu);
      bracket(mu, d);
    }
    *mu_out = mu;
    if (delta_n_out) *delta_n_out = d;
    if (iters_out) *iters_out = static_cast<int32_t>(hm.size());
    if (rho_out) std::memcpy(rho_out, rho.data(), P.nnz * sizeof(double));
  });
}

int ndrho_eigenstates(ndrho_ctx* ctx, int32_t struct_id, double xi, double eta, int32_t k, int32_t max_iter,
                      double tol, double* eps_out, double* c_out, int32_t* iters_out, double* resid_out) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    DevStruct& ds = ctx->get(struct_id);
    const Plan& P = ds.plan;
    const int64_t n = P.n;
    if (k < 1 || k > EIG_NR || k > n) fail(NDRHO_EINVAL, "k must be in [1, min(16, n)]");
    if (!std::isfinite(xi) || !(eta >= 0.0) || !std::isfinite(eta)) fail(NDRHO_EINVAL, "xi finite and eta >= 0 required");
    if (max_iter < 1 || !(tol > 0.0)) fail(NDRHO_EINVAL, "max_iter >= 1 and tol > 0 required");
    if (!eps_out) fail(NDRHO_EINVAL, "eps_out is required");
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    ctx->build_eigen_plan(ds);
    const DevStruct::EigenPlan& E = ds.eig;
    // device buffers of this call
    std::vector<void*> mem;
    auto dalloc = [&](size_t bytes) {
      void* p = nullptr;
      if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) {
        (void)hipGetLastError();
        fail(NDRHO_ENOMEM, "eigenstate buffers");
      }
      mem.push_back(p);
      return p;
    };
    struct Free {
      std::vector<void*>& m;
      ~Free() {
        for (void* p : m) (void)hipFree(p);
      }
    } free_guard{mem};
    constexpr int NB = 2 * EIG_NR;
    const size_t cvec = static_cast<size_t>(n) * EIG_NR * sizeof(double2);
    double2* y = static_cast<double2*>(dalloc(cvec));
    double2* z = static_cast<double2*>(dalloc(cvec));
    double2* z2 = static_cast<double2*>(dalloc(cvec));
    double2* x = static_cast<double2*>(dalloc(cvec));
    double2* w = static_cast<double2*>(dalloc(static_cast<size_t>(E.w_rows) * EIG_NR * sizeof(double2)));
    double* V = static_cast<double*>(dalloc(static_cast<size_t>(n) * NB * sizeof(double)));
    double* HV = static_cast<double*>(dalloc(static_cast<size_t>(n) * NB * sizeof(double)));
    double* SV = static_cast<double*>(dalloc(static_cast<size_t>(n) * NB * sizeof(double)));
    double* C = static_cast<double*>(dalloc(static_cast<size_t>(n) * EIG_NR * sizeof(double)));
    double* HC = static_cast<double*>(dalloc(static_cast<size_t>(n) * EIG_NR * sizeof(double)));
    double* SC = static_cast<double*>(dalloc(static_cast<size_t>(n) * EIG_NR * sizeof(double)));
    double* Yc = static_cast<double*>(dalloc(NB * EIG_NR * sizeof(double)));
    double* th = static_cast<double*>(dalloc(EIG_NR * sizeof(double)));
    const int nblk = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(256, (n + 255) / 256)));
    const int64_t chunk = (n + nblk - 1) / nblk;
    double* part = static_cast<double*>(dalloc(static_cast<size_t>(nblk) * NB * NB * sizeof(double)));
    double2* d_alpha = static_cast<double2*>(dalloc(sizeof(double2)));

    // factor X = alpha S - H, alpha = xi + i eta (upward sweep of one pole, FP64)
    const double2 alpha = make_double2(xi, eta);
    HIP_OK(hipMemcpyAsync(d_alpha, &alpha, sizeof(double2), hipMemcpyHostToDevice, st));
    ctx->ensure_ws(P, 1);
    HIP_OK(launch_init_acc(ds.m0, 0, 0, ctx->acc, ctx->status, st));
    ctx->run_pass(ds, 1, 0, 1, d_alpha, 0, 1.0, 0, 1, st, true);
    int stat[2];
    ctx->read_status(stat);
    if (stat[0]) fail(NDRHO_ESINGULAR, "a zero, tiny or non-finite pivot occurred in alpha S - H (use eta > 0)");

    // starting block: counter-based uniform numbers
    std::vector<double> h0(static_cast<size_t>(n) * EIG_NR);
    for (size_t i = 0; i < h0.size(); ++i) h0[i] = splitmix_uniform(i);
    HIP_OK(hipMemcpyAsync(C, h0.data(), h0.size() * sizeof(double), hipMemcpyHostToDevice, st));
    std::vector<double> hp(static_cast<size_t>(nblk) * NB * NB), hs(NB * NB), hh(NB * NB);
    std::vector<double> theta(EIG_NR, 0.0), res(EIG_NR, 0.0), ycoef(NB * EIG_NR, 0.0);
    auto gram = [&](const double* W, std::vector<double>& out) {
      HIP_OK(launch_gram(V, W, n, chunk, nblk, part, st));
      HIP_OK(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      for (int e = 0; e < NB * NB; ++e) {
        double acc = 0.0;
        for (int b = 0; b < nblk; ++b) acc += hp[static_cast<size_t>(b) * NB * NB + e];
        out[e] = acc;
      }
      for (int i = 0; i < NB; ++i)  // symmetrize the rounding
        for (int j = 0; j < i; ++j) out[i * NB + j] = out[j * NB + i] = 0.5 * (out[i * NB + j] + out[j * NB + i]);
    };
    int it = 0;
    bool done = false;
    std::vector<int> wanted;
    while (it < max_iter && !done) {
      ++it;
      // Eq. (B2): B = X^{-1} S C; the real basis V = [Re B, Im B]
      HIP_OK(launch_spmm_perm(E.rp, E.col, ds.s, E.perm, n, C, y, st));
      ctx->solve_factor(ds, y, z, z2, x, w);
      HIP_OK(launch_unperm_split(x, E.iperm, n, V, st));
      HIP_OK(launch_spmm2(E.rp, E.col, ds.h, n, V, HV, st));
      HIP_OK(launch_spmm2(E.rp, E.col, ds.s, n, V, SV, st));
      // Eq. (B3): <V|H|V> y = <V|S|V> y eps, with the S-metric's null
      // directions removed (canonical orthogonalization)
      gram(HV, hh);
      gram(SV, hs);
      std::vector<double> ls, us;
      sym_eig(NB, hs, ls, us);
      const double lmax = std::max(ls[NB - 1], 0.0);
      std::vector<int> keep;
      for (int i = 0; i < NB; ++i)
        if (ls[i] > 1e-13 * lmax) keep.push_back(i);
      const int r = static_cast<int>(keep.size());
      if (r == 0) fail(NDRHO_ESINGULAR, "the shift-invert block vanished");
      std::vector<double> W(static_cast<size_t>(NB) * r);  // NB x r, W = U_keep diag(l^-1/2)
      for (int i = 0; i < NB; ++i)
        for (int j = 0; j < r; ++j) W[i * r + j] = us[i * NB + keep[j]] / std::sqrt(ls[keep[j]]);
      std::vector<double> ht(static_cast<size_t>(r) * r, 0.0);  // W^T Hs W
      for (int a = 0; a < r; ++a)
        for (int b = 0; b < r; ++b) {
          double acc = 0.0;
          for (int i = 0; i < NB; ++i) {
            double t = 0.0;
            for (int j = 0; j < NB; ++j) t += hh[i * NB + j] * W[j * r + b];
            acc += W[i * r + a] * t;
          }
          ht[a * r + b] = acc;
        }
      for (int a = 0; a < r; ++a)
        for (int b = 0; b < a; ++b) ht[a * r + b] = ht[b * r + a] = 0.5 * (ht[a * r + b] + ht[b * r + a]);
      std::vector<double> lt, zt;
      sym_eig(r, ht, lt, zt);
      // the Ritz pairs nearest xi fill the next block (nearest first)
      std::vector<int> ord(r);
      for (int i = 0; i < r; ++i) ord[i] = i;
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return std::fabs(lt[a] - xi) < std::fabs(lt[b] - xi); });
      const int m = std::min(r, EIG_NR);
      std::fill(ycoef.begin(), ycoef.end(), 0.0);
      std::fill(theta.begin(), theta.end(), 0.0);
      for (int c = 0; c < m; ++c) {
        theta[c] = lt[ord[c]];
        for (int i = 0; i < NB; ++i) {
          double acc = 0.0;
          for (int j = 0; j < r; ++j) acc += W[i * r + j] * zt[j * r + ord[c]];
          ycoef[i * EIG_NR + c] = acc;
        }
      }
      HIP_OK(hipMemcpyAsync(Yc, ycoef.data(), ycoef.size() * sizeof(double), hipMemcpyHostToDevice, st));
      HIP_OK(hipMemcpyAsync(th, theta.data(), theta.size() * sizeof(double), hipMemcpyHostToDevice, st));
      HIP_OK(launch_combine(V, Yc, n, C, st));
      HIP_OK(launch_combine(HV, Yc, n, HC, st));
      HIP_OK(launch_combine(SV, Yc, n, SC, st));
      HIP_OK(launch_resid(HC, SC, th, n, chunk, nblk, part, st));
      std::vector<double> rp(static_cast<size_t>(nblk) * EIG_NR);
      HIP_OK(hipMemcpyAsync(rp.data(), part, rp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      for (int c = 0; c < EIG_NR; ++c) {
        double acc = 0.0;
        for (int b = 0; b < nblk; ++b) acc += rp[static_cast<size_t>(b) * EIG_NR + c];
        res[c] = std::sqrt(acc);
      }
      if (m < k) continue;  // not enough independent directions yet
      done = true;
      for (int c = 0; c < k; ++c) done = done && res[c] <= tol;
    }
    // the k Ritz pairs nearest xi, ascending in energy
    std::vector<int> pick(k);
    for (int c = 0; c < k; ++c) pick[c] = c;
    std::sort(pick.begin(), pick.end(), [&](int a, int b) { return theta[a] < theta[b]; });
    for (int c = 0; c < k; ++c) {
      eps_out[c] = theta[pick[c]];
      if (resid_out) resid_out[c] = res[pick[c]];
    }
    if (iters_out) *iters_out = it;
    if (c_out) {
      std::vector<double> hc(static_cast<size_t>(n) * EIG_NR);
      HIP_OK(hipMemcpyAsync(hc.data(), C, hc.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      for (int c = 0; c < k; ++c)
        for (int64_t i = 0; i < n; ++i) c_out[int64_t(c) * n + i] = hc[static_cast<size_t>(i) * EIG_NR + pick[c]];
    }
    HIP_OK(hipStreamSynchronize(st));
  });
}

int ndrho_set_shifts(ndrho_ctx* ctx, int32_t struct_id, int32_t n, const double* alpha_re, const double* alpha_im,
                     const double* weight, int32_t add_m0) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    DevStruct& ds = ctx->get(struct_id);
    if (n < 1 || !alpha_re || !alpha_im || !weight) fail(NDRHO_EINVAL, "n >= 1 and all arrays are required");
    std::vector<double2> a(n);
    std::vector<double> w(n);
    for (int k = 0; k < n; ++k) {
      if (!std::isfinite(alpha_re[k]) || !std::isfinite(alpha_im[k]) || !std::isfinite(weight[k]))
        fail(NDRHO_EINVAL, "non-finite shift or weight");
      a[k] = make_double2(alpha_re[k], alpha_im[k]);
      w[k] = weight[k];
    }
    HIP_OK(hipSetDevice(ctx->device));
    ctx->set_shifts(ds, a, w, add_m0 != 0, false);
  });
}

int ndrho_density_matrix_noalloc(ndrho_ctx* ctx, int32_t struct_id, double* rho_out_dev) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    DevStruct& ds = ctx->get(struct_id);
    if (!rho_out_dev) fail(NDRHO_EINVAL, "rho_out_dev is NULL");
    if (ds.n_shifts < 1) fail(NDRHO_ESTATE, "set_poles (or set_shifts) has not been called for this structure");
    HIP_OK(hipSetDevice(ctx->device));
    const Plan& P = ds.plan;
    // scratch layout: [status (256 B)][accumulator, nnz doubles, 256-aligned]
    // [workspace of nb poles]
    const size_t acc_bytes = (static_cast<size_t>(P.nnz) * sizeof(double) + 255) / 256 * 256;
    const size_t per_pole = static_cast<size_t>(ndrho_ctx::per_pole_elems(P)) * sizeof(double2);
    auto need = [&](int nb) {
      return 256 + acc_bytes + per_pole * size_t(nb);
    };
    if (need(1) > kScratchBytes)
      fail(NDRHO_ENOMEM, "the structure needs " + std::to_string(need(1)) +
                             " bytes of scratch for one pole; the no-allocation entry point holds " +
                             std::to_string(kScratchBytes));
    int nb = 1;
    while (nb < ds.n_shifts && need(nb + 1) <= kScratchBytes) ++nb;
    char* base = static_cast<char*>(ctx->scratch);
    // the evaluation runs on the scratch: one launch chain of plain launches
    // (no graph, no further streams), passes of nb poles
    struct Swap {
      ndrho_ctx* c;
      void* ws;
      size_t ws_bytes;
      double* acc;
      int64_t acc_len;
      int* status;
      ndrho_options opt;
      bool prof;
      ~Swap() {
        c->ws = ws, c->ws_bytes = ws_bytes, c->acc = acc, c->acc_len = acc_len, c->status = status, c->opt = opt;
        c->prof = prof;
      }
    } swap{ctx, ctx->ws, ctx->ws_bytes, ctx->acc, ctx->acc_len, ctx->status, ctx->opt, ctx->prof};
    ctx->status = reinterpret_cast<int*>(base);
    ctx->acc = reinterpret_cast<double*>(base + 256);
    ctx->acc_len = P.nnz;
    ctx->ws = base + 256 + acc_bytes;
    ctx->ws_bytes = per_pole * size_t(nb);
    ctx->opt.use_graph = 0;
    ctx->opt.split_streams = 0;
    ctx->opt.pole_batch = nb;
    ctx->prof = false;
    const auto t0 = std::chrono::steady_clock::now();
    ctx->evaluate(ds, ds.d_alpha, 0, ds.d_w, ds.n_shifts, ds.n_hi, ds.add_m0, 1.0, 0);
    HIP_OK(launch_scatter(ds.acc_entry, P.nnz, ctx->acc, rho_out_dev, ctx->stream));
    int st[2];
    ctx->read_status(st);
    if (st[0]) fail(NDRHO_ESINGULAR, "a zero, tiny or non-finite pivot occurred in alpha S - H");
    ctx->last_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  });
}

int ndrho_density_matrix(ndrho_ctx* ctx, int32_t struct_id, double* rho_out, int32_t on_device) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    DevStruct& ds = ctx->get(struct_id);
    if (!rho_out) fail(NDRHO_EINVAL, "rho_out is NULL");
    if (ds.n_shifts < 1) fail(NDRHO_ESTATE, "set_poles (or set_shifts) has not been called for this structure");
    HIP_OK(hipSetDevice(ctx->device));
    const auto t0 = std::chrono::steady_clock::now();
    const Plan& P = ds.plan;
    ctx->evaluate(ds, ds.d_alpha, 0, ds.d_w, ds.n_shifts, ds.n_hi, ds.add_m0, 1.0, 0);
    double* dst = on_device ? rho_out : ctx->outbuf;
    HIP_OK(launch_scatter(ds.acc_entry, P.nnz, ctx->acc, dst, ctx->stream));
    int st[2];
    ctx->read_status(st);
    if (st[0]) fail(NDRHO_ESINGULAR, "a zero, tiny or non-finite pivot occurred in alpha S - H");
    if (!on_device) {
      HIP_OK(hipMemcpyAsync(rho_out, ctx->outbuf, P.nnz * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      HIP_OK(hipStreamSynchronize(ctx->stream));
    }
    ctx->last_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  });
}

int ndrho_energy_density_matrix(ndrho_ctx* ctx, int32_t struct_id, double* rho_out, double* e_out,
                                int32_t on_device) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    DevStruct& ds = ctx->get(struct_id);
    if (!rho_out || !e_out) fail(NDRHO_EINVAL, "rho_out and e_out are required");
    if (ds.n_shifts < 1 || !ds.cf_poles) fail(NDRHO_ESTATE, "set_poles has not been called for this structure");
    HIP_OK(hipSetDevice(ctx->device));
    const auto t0 = std::chrono::steady_clock::now();
    const Plan& P = ds.plan;
    ctx->ensure_edm(P.nnz);
    if (!ds.m1_valid) ctx->compute_m1(ds);
    ctx->evaluate(ds, ds.d_alpha, 0, ds.d_w, ds.n_shifts, ds.n_hi, ds.add_m0, 1.0, 0, true);
    double* dst = on_device ? rho_out : ctx->outbuf;
    double* dst_e = on_device ? e_out : ctx->outbuf_e;
    HIP_OK(launch_scatter(ds.acc_entry, P.nnz, ctx->acc, dst, ctx->stream));
    HIP_OK(launch_scatter(ds.acc_entry, P.nnz, ctx->acc_e, dst_e, ctx->stream));
    int st[2];
    ctx->read_status(st);
    if (st[0]) fail(NDRHO_ESINGULAR, "a zero, tiny or non-finite pivot occurred in alpha S - H");
    if (!on_device) {
      HIP_OK(hipMemcpyAsync(rho_out, ctx->outbuf, P.nnz * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      HIP_OK(hipMemcpyAsync(e_out, ctx->outbuf_e, P.nnz * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      HIP_OK(hipStreamSynchronize(ctx->stream));
    }
    ctx->last_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  });
}

int ndrho_energy_density_matrix_batch(ndrho_ctx* ctx, const int32_t* struct_ids, int32_t k, double* const* rho_outs,
                                      double* const* e_outs, int32_t on_device) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    if (k < 1 || !struct_ids || !rho_outs || !e_outs) fail(NDRHO_EINVAL, "invalid batch arguments");
    for (int32_t i = 0; i < k; ++i)
      if (!rho_outs[i] || !e_outs[i]) fail(NDRHO_EINVAL, "an output pointer is NULL");
    std::vector<int32_t> ids(struct_ids, struct_ids + k);
    HIP_OK(hipSetDevice(ctx->device));
    const auto t0 = std::chrono::steady_clock::now();
    DevStruct& U = ctx->prepare_batch(ids);
    if (!U.cf_poles) fail(NDRHO_ESTATE, "set_poles has not been called for every batch member");
    const Plan& P = U.plan;
    const DevStruct& first = ctx->get(ids[0]);
    const int n = first.n_shifts;
    ctx->ensure_edm(P.nnz);
    if (!U.m1_valid) ctx->compute_m1(U);
    ctx->evaluate(U, U.d_alpha, n, U.d_w, n, first.n_hi, first.add_m0, 1.0, 0, true);
    HIP_OK(launch_scatter(U.acc_entry, P.nnz, ctx->acc, ctx->outbuf, ctx->stream));
    HIP_OK(launch_scatter(U.acc_entry, P.nnz, ctx->acc_e, ctx->outbuf_e, ctx->stream));
    int st[2];
    ctx->read_status(st);
    if (st[0]) fail(NDRHO_ESINGULAR, "a zero, tiny or non-finite pivot occurred in alpha S - H");
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    for (int32_t i = 0; i < k; ++i) {
      const int64_t cnt = ctx->get(ids[i]).plan.nnz;
      HIP_OK(hipMemcpyAsync(rho_outs[i], ctx->outbuf + P.struct_nnz_off[i], cnt * sizeof(double), kind, ctx->stream));
      HIP_OK(hipMemcpyAsync(e_outs[i], ctx->outbuf_e + P.struct_nnz_off[i], cnt * sizeof(double), kind, ctx->stream));
    }
    HIP_OK(hipStreamSynchronize(ctx->stream));
    ctx->last_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  });
}

int ndrho_density_matrix_batch(ndrho_ctx* ctx, const int32_t* struct_ids, int32_t k, double* const* rho_outs,
                               int32_t on_device) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    if (k < 1 || !struct_ids || !rho_outs) fail(NDRHO_EINVAL, "invalid batch arguments");
    for (int32_t i = 0; i < k; ++i)
      if (!rho_outs[i]) fail(NDRHO_EINVAL, "rho_outs has a NULL entry");
    std::vector<int32_t> ids(struct_ids, struct_ids + k);
    HIP_OK(hipSetDevice(ctx->device));
    const auto t0 = std::chrono::steady_clock::now();
    DevStruct& U = ctx->prepare_batch(ids);
    const Plan& P = U.plan;
    const DevStruct& first = ctx->get(ids[0]);
    const int n = first.n_shifts;
    ctx->evaluate(U, U.d_alpha, n, U.d_w, n, first.n_hi, first.add_m0, 1.0, 0);
    HIP_OK(launch_scatter(U.acc_entry, P.nnz, ctx->acc, ctx->outbuf, ctx->stream));
    int st[2];
    ctx->read_status(st);
    if (st[0]) fail(NDRHO_ESINGULAR, "a zero, tiny or non-finite pivot occurred in alpha S - H");
    for (int32_t i = 0; i < k; ++i) {
      const int64_t cnt = ctx->get(ids[i]).plan.nnz;
      HIP_OK(hipMemcpyAsync(rho_outs[i], ctx->outbuf + P.struct_nnz_off[i], cnt * sizeof(double),
                            on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->stream));
    }
    HIP_OK(hipStreamSynchronize(ctx->stream));
    ctx->last_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  });
}

int ndrho_autotune(ndrho_ctx* ctx, const int32_t* struct_ids, int32_t k, const char* cache_path) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    if (k < 1 || !struct_ids) fail(NDRHO_EINVAL, "invalid structure list");
    HIP_OK(hipSetDevice(ctx->device));
    std::vector<int32_t> ids(struct_ids, struct_ids + k);
    DevStruct& T = k == 1 ? ctx->get(ids[0]) : ctx->prepare_batch(ids);
    if (T.n_shifts < 1) fail(NDRHO_ESTATE, "set_poles (or set_shifts) has not been called");
    const Plan& P = T.plan;
    const int nops = static_cast<int>(P.upward.size() + P.downward.size());
    const int nb = ctx->batch_for(P, T.n_shifts);
    char keybuf[256];
    std::snprintf(keybuf, sizeof(keybuf),
                  "ndrho-tune-v6 n=%lld nnz=%lld fronts=%zu shifts=%d fp64=%d batch=%d prec=%d piv=%d ops=%d",
                  static_cast<long long>(P.n), static_cast<long long>(P.nnz), P.fronts.size(), T.n_shifts, T.n_hi,
                  nb, ctx->opt.precision, ctx->opt.pivot_variant, nops);
    const std::string key(keybuf);
    // the launches whose variant is chosen here: front updates unless
    // gemm_variant forces one, pivot-inverse products unless pivot_variant does
    auto tunable = [&](const Op& op) {
      return op.kind == OP_GEMM && ((op.flags & OP_PIVOT) ? ctx->opt.pivot_variant < 0 : ctx->opt.gemm_variant < 0);
    };
    bool any = false;
    for (const Op& op : P.upward) any = any || tunable(op);
    for (const Op& op : P.downward) any = any || tunable(op);
    if (T.n_hi >= T.n_shifts || !any) return;  // nothing to choose
    if (cache_path) {
      std::ifstream in(cache_path);
      std::string line;
      while (std::getline(in, line)) {
        if (line.size() != key.size() + 1 + static_cast<size_t>(nops) || line.compare(0, key.size(), key) != 0 ||
            line[key.size()] != ' ')
          continue;
        // a line is used only if every digit is a variant this precision mode accepts
        std::vector<int8_t> v(nops);
        bool ok = true;
        for (int i = 0; i < nops && ok; ++i) {
          const int d = line[key.size() + 1 + i] - '0';
          ok = d >= 0 && d < V_COUNT && variant_allowed(ctx->opt.precision, d);
          v[i] = static_cast<int8_t>(d);
        }
        if (!ok) continue;
        T.variant = v;
        ++T.tune_gen;
        return;
      }
    }
    // time every variant of every tunable GEMM launch on one full evaluation each
    std::vector<std::vector<double>> ms(V_COUNT, std::vector<double>(nops, 0.0));
    const bool was_prof = ctx->prof;
    const std::vector<int8_t> saved = T.variant;
    const int64_t astride = k == 1 ? 0 : T.n_shifts;
    try {
      for (int v = 0; v < V_COUNT; ++v) {
        if (!variant_allowed(ctx->opt.precision, v)) continue;
        for (int i = 0; i < nops; ++i) {
          const Op& op = i < static_cast<int>(P.upward.size()) ? P.upward[i] : P.downward[i - P.upward.size()];
          T.variant[i] = tunable(op) ? static_cast<int8_t>(v) : int8_t(V_FP64);
        }
        ctx->prof = true;
        ctx->op_ms = &ms[v];
        ctx->evaluate(T, T.d_alpha, astride, T.d_w, T.n_shifts, T.n_hi, T.add_m0, 1.0, 0);
        int st[2];
        ctx->read_status(st);
        ctx->op_ms = nullptr;
        if (ctx->opt.verbose) {
          double tot = 0;
          for (double x : ms[v]) tot += x;
          std::fprintf(stderr, "ndrho_autotune: variant %d timed, %.1f ms of launches\n", v, tot);
        }
      }
    } catch (...) {
      ctx->op_ms = nullptr;
      ctx->prof = was_prof;
      T.variant = saved;
      throw;
    }
    ctx->prof = was_prof;
    ctx->clear_profile();
    std::string choice;
    for (int i = 0; i < nops; ++i) {
      const Op& op = i < static_cast<int>(P.upward.size()) ? P.upward[i] : P.downward[i - P.upward.size()];
      int best = V_FP64;  // only the tunable GEMM launches have variants
      if (tunable(op))
        for (int v = 1; v < V_COUNT; ++v)
          if (variant_allowed(ctx->opt.precision, v) && ms[v][i] < ms[best][i]) best = v;
      T.variant[i] = static_cast<int8_t>(best);
      choice.push_back(static_cast<char>('0' + best));
    }
    ++T.tune_gen;
    if (ctx->opt.verbose) std::fprintf(stderr, "ndrho_autotune: choice per launch %s\n", choice.c_str());
    if (cache_path) {
      std::ofstream out(cache_path, std::ios::app);
      out << key << ' ' << choice << '\n';
    }
  });
}

int ndrho_structure_stats(const ndrho_ctx* ctx, int32_t struct_id, ndrho_stats_t* out) {
  if (!ctx || !out) return NDRHO_EINVAL;
  ndrho_ctx* c = const_cast<ndrho_ctx*>(ctx);
  return guarded(c, [&] {
    DevStruct& ds = c->get(struct_id);
    const Plan& P = ds.plan;
    std::memset(out, 0, sizeof(*out));
    out->n = P.n;
    out->nnz = P.nnz;
    out->n_fronts = static_cast<int32_t>(P.fronts.size());
    out->n_levels = P.n_levels;
    for (const Front& F : P.fronts) {
      out->max_front_j = std::max(out->max_front_j, F.nj);
      out->max_front_u = std::max(out->max_front_u, F.nu);
      if (F.parent < 0) out->root_j = std::max(out->root_j, F.nj);
    }
    out->n_poles = ds.n_shifts;
    out->pole_batch = c->last_batch;
    out->flops_per_pole = P.flops_model;
    out->flops_exec_per_pole = P.flops_exec;
    out->bytes_per_pole = P.bytes_model;
    out->factor_bytes_per_pole = static_cast<double>(P.panel_total) * sizeof(double2);
    out->workspace_bytes = static_cast<double>(c->ws_bytes);
    out->last_ms = c->last_ms;
    out->launches_per_pass = static_cast<int64_t>(P.upward.size() + P.downward.size() + 1);
    out->n_fp64_poles = ds.n_hi;
    out->split_passes = ds.split_passes;
    out->precision = c->opt.precision;
  });
}

int ndrho_stats(const ndrho_ctx* ctx, double* ms_per_phase, double* flops, double* hbm_bytes) {
  if (!ctx) return NDRHO_EINVAL;
  if (ms_per_phase)
    for (int k = 0; k < 4; ++k) ms_per_phase[k] = ctx->prof_phase_ms[k];
  if (flops) *flops = ctx->last_flops;
  if (hbm_bytes) *hbm_bytes = ctx->last_bytes;
  return NDRHO_OK;
}

int ndrho_profile(ndrho_ctx* ctx, int32_t enable) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    HIP_OK(hipStreamSynchronize(ctx->stream));
    if (!ctx->recs.empty()) ctx->fold_profile();
    ctx->prof = enable != 0;
    if (ctx->prof) ctx->clear_profile();
  });
}

int ndrho_profile_read(const ndrho_ctx* ctx, double* ms, double* flops, int64_t* launches) {
  if (!ctx) return NDRHO_EINVAL;
  for (int k = 0; k < NDRHO_K_COUNT; ++k) {
    if (ms) ms[k] = ctx->prof_ms[k];
    if (flops) flops[k] = ctx->prof_flops[k];
    if (launches) launches[k] = ctx->prof_n[k];
  }
  return NDRHO_OK;
}

int ndrho_profile_read_bytes(const ndrho_ctx* ctx, double* bytes) {
  if (!ctx || !bytes) return NDRHO_EINVAL;
  for (int k = 0; k < NDRHO_K_COUNT; ++k) bytes[k] = ctx->prof_bytes[k];
  return NDRHO_OK;
}

int ndrho_profile_read_depth(const ndrho_ctx* ctx, double* ms) {
  if (!ctx || !ms) return NDRHO_EINVAL;
  for (int i = 0; i < NDRHO_K_COUNT * NDRHO_PROFILE_DEPTHS; ++i) ms[i] = ctx->prof_depth_ms[i];
  return NDRHO_OK;
}

int ndrho_device_alloc(ndrho_ctx* ctx, int64_t bytes, void** ptr) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    if (!ptr || bytes <= 0) fail(NDRHO_EINVAL, "bytes must be positive and ptr non-NULL");
    HIP_OK(hipSetDevice(ctx->device));
    *ptr = nullptr;
    if (hipMalloc(ptr, static_cast<size_t>(bytes)) != hipSuccess) {
      (void)hipGetLastError();
      fail(NDRHO_ENOMEM, "device allocation failed");
    }
  });
}

int ndrho_device_free(ndrho_ctx* ctx, void* ptr) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    if (!ptr) return;
    HIP_OK(hipSetDevice(ctx->device));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    HIP_OK(hipFree(ptr));
  });
}

int ndrho_device_to_host(ndrho_ctx* ctx, void* dst, const void* src, int64_t bytes) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    if (!dst || !src || bytes < 0) fail(NDRHO_EINVAL, "invalid copy arguments");
    HIP_OK(hipSetDevice(ctx->device));
    HIP_OK(hipMemcpyAsync(dst, src, static_cast<size_t>(bytes), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
  });
}

int ndrho_device_copy(ndrho_ctx* ctx, void* dst, const void* src, int64_t bytes) {
  if (!ctx) return NDRHO_EINVAL;
  return guarded(ctx, [&] {
    if (!dst || !src || bytes < 0 || bytes % 16) fail(NDRHO_EINVAL, "invalid copy arguments");
    HIP_OK(hipSetDevice(ctx->device));
    HIP_OK(launch_stream_copy(src, dst, bytes, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
  });
}

int ndrho_cf_poles(int32_t n_poles, double* z, double* R) {
  return guarded(nullptr, [&] {
    if (!z || !R) fail(NDRHO_EINVAL, "z and R are required");
    cf_poles(n_poles, z, R);
  });
}

int ndrho_plan_create(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* coords,
                      const double* cell, int32_t leaf_rows, double long_tail, ndrho_plan** out) {
  return guarded(nullptr, [&] {
    if (!out) fail(NDRHO_EINVAL, "out is NULL");
    *out = nullptr;
    validate_csr(n, row_ptr, col_idx, nullptr, nullptr);
    if (cell && !coords) fail(NDRHO_EINVAL, "a periodic cell needs the coordinates");
    std::unique_ptr<ndrho_plan> p(new ndrho_plan());
    build_plan(p->plan, n, row_ptr, col_idx, coords, leaf_rows, long_tail, cell);
    *out = p.release();
  });
}

int ndrho_plan_destroy(ndrho_plan* plan) {
  delete plan;
  return NDRHO_OK;
}

const char* ndrho_plan_last_error(void) { return g_err.c_str(); }

int ndrho_plan_counts(const ndrho_plan* plan, int64_t* counts) {
  if (!plan || !counts) return NDRHO_EINVAL;
  const Plan& P = plan->plan;
  int64_t su = 0, mj = 0, mu = 0;
  for (const Front& F : P.fronts) {
    su += F.nu;
    mj = std::max<int64_t>(mj, F.nj);
    mu = std::max<int64_t>(mu, F.nu);
  }
  counts[0] = static_cast<int64_t>(P.fronts.size());
  counts[1] = P.n_levels;
  counts[2] = su;
  counts[3] = P.nnz;
  counts[4] = P.panel_total;
  counts[5] = mj;
  counts[6] = mu;
  return NDRHO_OK;
}

int ndrho_plan_export(const ndrho_plan* plan, int32_t* perm, int32_t* parent, int32_t* depth, int64_t* j0,
                      int32_t* nj, int32_t* nu, int64_t* u_off, int32_t* u_rows, int32_t* rel) {
  if (!plan) return NDRHO_EINVAL;
  const Plan& P = plan->plan;
  if (perm) std::memcpy(perm, P.perm.data(), P.n * sizeof(int32_t));
  int64_t off = 0;
  for (size_t f = 0; f < P.fronts.size(); ++f) {
    const Front& F = P.fronts[f];
    if (parent) parent[f] = F.parent;
    if (depth) depth[f] = F.depth;
    if (j0) j0[f] = F.j0;
    if (nj) nj[f] = F.nj;
    if (nu) nu[f] = F.nu;
    if (u_off) u_off[f] = off;
    for (int k = 0; k < F.nu; ++k) {
      if (u_rows) u_rows[off + k] = F.u[k];
      if (rel) rel[off + k] = F.parent >= 0 ? F.rel[k] : -1;
    }
    off += F.nu;
  }
  return NDRHO_OK;
}

int ndrho_plan_slots(const ndrho_plan* plan, int64_t* out_slot, int64_t* asm_slot, int64_t* panel_off) {
  if (!plan) return NDRHO_EINVAL;
  const Plan& P = plan->plan;
  if (out_slot) std::memcpy(out_slot, P.out_slot.data(), P.nnz * sizeof(int64_t));
  if (asm_slot) std::memcpy(asm_slot, P.asm_slot.data(), P.nnz * sizeof(int64_t));
  if (panel_off)
    for (size_t f = 0; f < P.fronts.size(); ++f) panel_off[f] = P.fronts[f].panel_off;
  return NDRHO_OK;
}

int ndrho_plan_program(const ndrho_plan* plan, int64_t* count, int32_t* kind, int32_t* depth, double* flops,
                       int64_t* items) {
  if (!plan || !count) return NDRHO_EINVAL;
  const Plan& P = plan->plan;
  int64_t i = 0;
  auto put = [&](const Op& op) {
    static const int kmap[] = {NDRHO_K_EXTADD, NDRHO_K_ASSEMBLE, NDRHO_K_PIVOT_INV, NDRHO_K_GEMM,
                               NDRHO_K_COPY,   NDRHO_K_GATHER,   NDRHO_K_SMALL};
    if (kind) kind[i] = kmap[op.kind];
    if (depth) depth[i] = op.depth;
    if (flops) flops[i] = op.flops;
    if (items) items[i] = op.tile_count ? op.tile_count : op.count;
    ++i;
  };
  for (const Op& op : P.upward) put(op);
  for (const Op& op : P.downward) put(op);
  *count = i;
  return NDRHO_OK;
}

int ndrho_plan_model(const ndrho_plan* plan, double* flops, double* bytes) {
  if (!plan) return NDRHO_EINVAL;
  if (flops) *flops = plan->plan.flops_model;
  if (bytes) *bytes = plan->plan.bytes_model;
  return NDRHO_OK;
}

}  // extern "C"
