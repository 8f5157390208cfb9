// C ABI (include/qtn.h): network build, planning, schedule and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "device.hpp"
#include "kernels.hpp"
#include "mlp.hpp"
#include "plan.hpp"
#include "qtn.h"

using namespace qtn;

namespace {

thread_local std::string g_err;

int set_err(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define QTN_HIP(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return set_err(QTN_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Status of the exception being handled, at the C ABI, which no C++
// exception crosses: QTN_ENOMEM for a failed host allocation, QTN_EINVAL
// ("internal error: ...") for anything else.
int exception_status() {
  try {
    throw;
  } catch (const std::bad_alloc &) {
    return set_err(QTN_ENOMEM, "host allocation failed");
  } catch (const std::exception &e) {
    return set_err(QTN_EINVAL, std::string("internal error: ") + e.what());
  } catch (...) {
    return set_err(QTN_EINVAL, "internal error");
  }
}

uint32_t pext32(uint32_t x, uint32_t mask) {
  uint32_t r = 0, d = 0;
  for (int b = 0; b < 32; b++)
    if ((mask >> b) & 1u) r |= ((x >> b) & 1u) << d++;
  return r;
}

// Runs f(i) for i in [0, n) on up to hardware_concurrency threads.
template <class F>
void parallel_for(int n, F f) {
  int nt = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 32u);
  nt = std::min(nt, n);
  if (nt <= 1) {
    for (int i = 0; i < n; i++) f(i);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (int t = 0; t < nt; t++)
    th.emplace_back([&] {
      for (int i = next++; i < n; i = next++) f(i);
    });
  for (auto &x : th) x.join();
}

struct Task {
  int kind;        // QTN_K_BLOCK: range index; QTN_K_WIDE: group index
  int index;
  uint32_t n_units;
  int variant;     // wide groups: mapping variant
  double bytes, flops;
};

// Device layout and launch list of one or more planned networks.
struct Schedule {
  int prec = 0;        // QTN_C128, QTN_C64 or QTN_MIXED
  int scalar_prec = 0;  // storage of the scalar slots
  std::vector<DevGroup> groups;
  std::vector<DevOp> ops;
  std::vector<int2> ranges;  // first n_cones: each cone's leading small groups
  std::vector<int> csb, ncb;
  std::vector<int> cns;       // slices per light cone (index slicing; 1: none)
  // hybrid executor: cones whose groups after the leading segment run by
  // per-group launches after the persistent launch (they may take the cell
  // mapping)
  std::vector<char> cone_heavy;
  std::vector<FillDesc> fills;
  std::vector<int32_t> stab;  // serial-offset tables of streaming operands
  std::vector<uint8_t> uperm; // 32 bytes per group: union bit of each unit bit
  std::vector<int> group_cone, group_index;  // plan position of each group
  std::vector<int> singles;   // groups also given a one-group range (tuning)
  int singles_range0 = 0;     // range index of singles[0]
  std::vector<std::vector<Task>> cone_tasks;  // after the leading small groups
  int n_cones = 0, n_nets = 0, n_angles = 0;
  size_t off_res = 0, off_angles = 0, off_desc = 0, off_fills = 0, off_groups = 0,
         off_ops = 0, off_stab = 0, off_uperm = 0, off_ranges = 0, off_csb = 0, off_ncb = 0, off_cns = 0, off_data = 0, total = 0;
  int64_t scalar_off = 0, scalar_sstride = 0;
  int n_sets = 1;  // angle sets evaluated per launch (one copy of the data each)
  std::vector<char> desc_blob;  // bytes [off_desc, off_data)
  uint64_t serial = 0;          // distinct for every schedule built
  int item_order = 0;           // lockstep steps: 0 costliest cone's items first, 1 reversed
  double bytes[QTN_NKERNELS] = {}, flops[QTN_NKERNELS] = {};
  double init_bytes = 0, init_flops = 0;
  // persistent executors: work items in step order; the task (one cone's
  // segment or wide group) of each item, each task's predecessor in its cone
  // (-1: none) and its item count
  std::vector<int4> items;
  std::vector<int> step_begin, item_task, task_dep, task_need, task_next, task_first;
  int n_steps = 0, n_tasks = 0, n_init = 0;
  size_t off_items = 0, off_steps = 0, off_item_task = 0, off_task_next = 0, off_task_first = 0,
         off_task_need = 0, off_queue = 0, off_ctl = 0;
  int n_ctl = 0;
};

// Streams, events, pinned staging and the captured graph of one schedule.
struct Runtime {
  int device = -1;
  hipStream_t main = nullptr;
  std::vector<hipStream_t> side;
  hipEvent_t ev_in = nullptr, ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  double *pinned = nullptr;
  size_t pinned_n = 0;
  void *ws = nullptr;  // workspace the captured graph was recorded for
  // pinned copy of the schedule's descriptor bytes, uploaded into the
  // workspace before every evaluation (the workspace contents are the
  // caller's between calls, and other schedules may share its address)
  char *pinned_desc = nullptr;
  size_t pinned_desc_cap = 0, pinned_desc_n = 0;
  uint64_t desc_serial = 0;  // schedule whose blob the pinned copy holds
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int persist_blocks = 0;
  uint32_t *pinned_err = nullptr;

  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    for (auto s : side) (void)hipStreamDestroy(s);
    side.clear();
    for (auto e : ev_join) (void)hipEventDestroy(e);
    ev_join.clear();
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (main) (void)hipStreamDestroy(main);
    if (pinned) (void)hipHostFree(pinned);
    if (pinned_err) (void)hipHostFree(pinned_err);
    if (pinned_desc) (void)hipHostFree(pinned_desc);
    pinned_err = nullptr;
    pinned_desc = nullptr;
    pinned_desc_cap = pinned_desc_n = 0;
    desc_serial = 0;
    persist_blocks = 0;
    ev_in = ev_fork = nullptr;
    main = nullptr;
    pinned = nullptr;
    pinned_n = 0;
    ws = nullptr;
    device = -1;
  }
  // The captured graph and the uploaded descriptors belong to one schedule.
  void forget_schedule() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    ws = nullptr;
    desc_serial = 0;
    pinned_desc_n = 0;
  }
  // Takes over o's streams, events and pinned buffers (o is left empty), for
  // a new schedule of the same network: streams are not torn down and
  // re-created when a plan is re-tuned.
  void take(Runtime &o) {
    if (&o == this) return;
    release();
    device = o.device;
    main = o.main;
    side.swap(o.side);
    ev_in = o.ev_in;
    ev_fork = o.ev_fork;
    ev_join.swap(o.ev_join);
    pinned = o.pinned;
    pinned_n = o.pinned_n;
    persist_blocks = o.persist_blocks;
    pinned_err = o.pinned_err;
    pinned_desc = o.pinned_desc;
    pinned_desc_cap = o.pinned_desc_cap;
    exec = o.exec;
    graph = o.graph;
    o.exec = nullptr;
    o.graph = nullptr;
    o.main = nullptr;
    o.ev_in = o.ev_fork = nullptr;
    o.pinned = nullptr;
    o.pinned_n = 0;
    o.pinned_err = nullptr;
    o.pinned_desc = nullptr;
    o.pinned_desc_cap = o.pinned_desc_n = 0;
    o.desc_serial = 0;
    o.persist_blocks = 0;
    o.ws = nullptr;
    o.device = -1;
    forget_schedule();
  }
  Runtime() = default;
  Runtime(const Runtime &) = delete;
  Runtime &operator=(const Runtime &) = delete;
  ~Runtime() { release(); }
};

struct Exec {
  Schedule sched;
  Runtime rt;
  bool persistent = false;
  bool dataflow = false;  // persistent: per-task dependencies instead of lockstep
  bool hybrid = false;    // persistent lockstep for light cones, launches for heavy ones
  bool lead_per_cone = false;
  uint32_t spin_limit = 1u << 22;
  int grid_quarters = 4;  // persistent grid: this many quarters of the resident blocks
};

std::atomic<uint64_t> g_sched_serial{0};  // Schedule::serial source

}  // namespace

struct qtn_network {
  Graph g;
  int p = 0;
  std::vector<double> gamma, beta;
  PlanOptions opt;
  int n_streams = 4;
  bool eager = false;
  int lane_sum_bits = 2;  // streaming: summed bits spread over lanes
  int order_trials = 0;   // >1: best of this many randomized min-fill orders
  int hybrid_width = 20;  // executor 5: cones with a bucket wider than this are heavy
  int executor = 0;       // 0 streams + per-group launches, 1 persistent lockstep
  uint32_t spin_limit = 1u << 22;
  int variant = 0;        // 0 auto, 1 generic only, 2 streaming where possible,
                          // 3 matrix form where possible, 4 cells where possible
  std::vector<LightCone> cones;
  std::vector<std::vector<int>> minfill;
  std::mutex minfill_lock;
  bool planned = false;
  int precision = 0;
  uint64_t version = 0;
  std::vector<ConePlan> plans;
  std::unique_ptr<Exec> exec;
  std::vector<qtn_launch_rec> launch_log;
  std::vector<qtn_tune_rec> tune_log;
  size_t tune_workspace = 0;
  // angle-set batches: a schedule with one data copy per set, rebuilt when
  // the set count or the plan changes
  std::unique_ptr<Exec> angle_exec;
  int angle_sets = 0;
  uint64_t angle_version = 0;
};

namespace {

std::mutex g_batch_lock;
std::map<std::vector<std::pair<const qtn_network *, uint64_t>>, std::unique_ptr<Exec>> g_batch;

void drop_batches_with(const qtn_network *net) {
  std::lock_guard<std::mutex> lk(g_batch_lock);
  for (auto it = g_batch.begin(); it != g_batch.end();) {
    bool has = false;
    for (auto &kv : it->first) has |= kv.first == net;
    it = has ? g_batch.erase(it) : std::next(it);
  }
}

const std::vector<int> &get_minfill(qtn_network *net, int e) {
  std::lock_guard<std::mutex> lk(net->minfill_lock);
  if (net->minfill[e].empty()) net->minfill[e] = minfill_order(net->cones[e]);
  return net->minfill[e];
}

// Element offset of a gate's values in the gate table.  A gate cut by index
// slicing reads the block whose bit 0 is its remaining axis, at the row of
// the fixed axis's value (bit cut_slot of the slice number).
int64_t gate_offset(const Gate &gt, bool transposed, int p, uint32_t slice = 0) {
  int t = transposed ? 4 : 0;
  if (gt.cut >= 0) t = (gt.cut == 1 ? 4 : 0) + 2 * (int)((slice >> gt.cut_slot) & 1u);
  switch (gt.kind) {
    case kH: return 32LL * p;
    case kZ: return 32LL * p + 2;
    case kP: return 32LL * gt.layer + 0 + t;
    case kPc: return 32LL * gt.layer + 8 + t;
    case kR: return 32LL * gt.layer + 16 + t;
    default: return 32LL * gt.layer + 24 + t;
  }
}

// Bytes of the largest operand of a group (gate tables count in the group's
// precision).  The streaming and cell mappings address the lane and cell
// parts of an operand with 32-bit byte offsets, so they take only groups
// whose operands all fit in 4 GiB; the generic mapping addresses elements
// with 64-bit indices and takes any group.
double max_operand_bytes(const Group &G, const ConePlan &pl) {
  double mx = 0;
  for (const Operand &o : G.ops) {
    const Tensor &t = pl.tensors[o.tensor];
    const int prec = t.gate >= 0 ? G.prec : t.prec;
    mx = std::max(mx, std::ldexp(prec == 1 ? 8.0 : 16.0, (int)t.vars.size()));
  }
  return mx;
}
constexpr double kOffset32Bytes = 4294967296.0;

// Candidate kernel configuration the autotuner forces on every wide group.
struct Force {
  int place;    // -1 keep, 0 workgroup segment, 1 own launch
  int variant;  // 1 generic, 2 streaming, 3 matrix form, 4 cells
  int rls;      // streaming: lane-summed bits; cells: register bits
};

constexpr int kTuneSingleWidth = 16;

// Configurations measured by the autotuner: every group in its own launch
// with the generic mapping, with the streaming mapping at 1, 2, 3
// lane-summed bits, in matrix form (groups that have one), or with
// the cell mapping at 3 or 4 cell bits (groups wide enough for it; 2 cell
// bits were measured too and never won on the N=30 p=4 network).
const std::vector<Force> &tune_candidates() {
  static const std::vector<Force> c = {{1, 1, 2}, {1, 2, 1}, {1, 2, 2}, {1, 2, 3},
                                       {1, 3, 2}, {1, 4, 3}, {1, 4, 4}};
  return c;
}

// Where a group's operands and output live (bytes from the data base) and
// the kernel configuration requested for it.
struct GroupEnv {
  int64_t out_off = 0, out_sstride = 0;   // output (tensor or scalar slot), set 0
  int64_t arena = 0, arena_sstride = 0;   // intermediates sit at arena + Tensor::offset
  int64_t table[2] = {-1, -1};            // gate tables: complex128, complex64
  int64_t table_sstride[2] = {0, 0};
  const std::vector<Gate> *gates = nullptr;  // gates of the group's gate operands
  uint32_t slice = 0;                     // index slicing: the slice's number
  int p = 0;                              // QAOA depth (gate table layout)
  int var_req = 0, rls_req = 2;           // mapping requested (0: the width rule)
  bool is_small = false;                  // runs inside a workgroup segment
  bool persistent = false;                // the schedule runs in a persistent executor
};

// Device descriptor of one group: chooses its mapping, appends its operands
// to s.ops (their tables to s.stab, its unit-bit order to s.uperm) and
// returns the group record with its algorithmic bytes and flops.
int describe_group(const Group &G, const ConePlan &pl, const GroupEnv &env, Schedule &s,
                   DevGroup *dg_out, double *bytes_out, double *flops_out) {
  auto es = [](int prec) { return prec == 1 ? (int64_t)8 : (int64_t)16; };
  DevGroup dg;
  std::memset(&dg, 0, sizeof dg);
  dg.out_off = env.out_off;
  dg.out_sstride = env.out_sstride;
  dg.prec = (uint8_t)G.prec;
  dg.op_begin = (int32_t)s.ops.size();
  dg.w = (uint8_t)G.w;
  dg.L = (uint8_t)G.L;
  dg.n_ops = (uint8_t)G.ops.size();
  double in_bytes = 0;
  std::vector<int> per_level(G.L, 0);
  for (const Operand &o : G.ops) {
    per_level[o.level]++;
    const Tensor &t = pl.tensors[o.tensor];
    in_bytes += std::ldexp(1.0, (int)t.vars.size()) * es(t.gate >= 0 ? G.prec : t.prec);
  }
  int var_req = env.var_req, rls_req = env.rls_req;
  const bool is_small = env.is_small, persistent = env.persistent;
  const int rls = std::min(G.L - 1, rls_req);
  const int sl = G.L - 1 - rls;
  const bool off32 = max_operand_bytes(G, pl) <= kOffset32Bytes;
  const bool stream_ok = (int)G.ops.size() <= kStreamMaxOps && sl <= kStreamMaxSerial && off32;
  // matrix form: groups that split into two sides (gemm_shape), requested or
  // picked by tuning; complex128 tiles take more LDS than the workgroup and
  // persistent kernels hold, so complex128 groups take it in own launches only
  GemmShape gsh;
  const bool mfma = var_req == 3 && (G.prec == 1 || (!is_small && !persistent)) &&
                    gemm_shape(G, pl, &gsh);
  if (var_req == 3 && !mfma) var_req = 0;
  // cells: lanes on union bits 0..5, cb cell bits in registers (the
  // summed bits above bit 5, then rb kept bits); own launches only (the
  // kernel is not part of the workgroup and persistent paths).  Taken
  // when requested, and by the rule for every own-launch group it fits
  const int low = std::max(G.L, 6);
  auto cell_fits = [&](int cbits) {
    const int r = cbits - std::max(0, G.L - 6);
    return !is_small && !persistent && off32 && (int)G.ops.size() <= 64 &&
           cell_lds_words((int)G.ops.size(), cbits) <= kCellMaxLdsWords &&
           G.L - 6 <= kCellMaxSerial && r >= 0 && G.w - low >= r;
  };
  int cb = 0;
  bool cell = false;
  if (var_req == 4) {
    cb = rls_req >= kCellMinCB && rls_req <= kCellMaxCB ? rls_req : kCellRuleCB;
    cell = cell_fits(cb);
    if (!cell) var_req = 0;
  }
  if (var_req == 0 && !mfma && cell_fits(kCellRuleCB)) {
    cb = kCellRuleCB;
    cell = true;
  }
  const int rb = cell ? cb - std::max(0, G.L - 6) : 0;
  // otherwise the streaming mapping once a lane walks >= 2 serial bits
  const bool stream =
      !mfma && !cell && stream_ok && (var_req == 2 || (var_req == 0 && sl >= 2));
  std::vector<int> order(G.ops.size());
  std::vector<int> cls(G.ops.size(), 0);
  for (size_t k = 0; k < G.ops.size(); k++) order[k] = (int)k;
  if (mfma) {
    dg.variant = kVarMfma;
    // [side A..., side B...]
    std::vector<int> side[2];
    for (int k = 0; k < (int)G.ops.size(); k++) side[gsh.role[k]].push_back(k);
    order.clear();
    for (auto &sd : side) order.insert(order.end(), sd.begin(), sd.end());
    dg.n_unit = (uint8_t)side[0].size();
    dg.n_step = (uint8_t)side[1].size();
    dg.n_serial = 0;
    dg.n_mb = (uint8_t)gsh.mbits.size();
    dg.n_nb = (uint8_t)gsh.nbits.size();
    dg.n_bb = (uint8_t)gsh.bbits.size();
    // column blocks of 16 per tile: as many as the n range fills (n >= 4
    // bits) in own launches; one inside workgroups and the persistent
    // executors, whose kernels are compiled for that form only
    dg.rls = (uint8_t)(is_small || persistent ? 1 : (dg.n_nb >= 6 ? 4 : (dg.n_nb == 5 ? 2 : 1)));
    const uint64_t tn = 16ull * dg.rls;
    const uint64_t mt = ((1ull << dg.n_mb) + kMmTM - 1) / kMmTM;
    const uint64_t nt = ((1ull << dg.n_nb) + tn - 1) / tn;
    const uint64_t tiles = (1ull << dg.n_bb) * mt * nt;
    if (tiles > 0xFFFFFFFFull) return set_err(QTN_ERANGE, "matrix-form group too large");
    dg.n_units = (uint32_t)tiles;
    // the tile's rows and columns: union bits of the lowest 6 m (n) bits
    dg.gtab = (int32_t)s.stab.size();
    for (int pass = 0; pass < 2; pass++) {
      const std::vector<int> &bl = pass == 0 ? gsh.mbits : gsh.nbits;
      const int lim = pass == 0 ? kMmTM : kMmTN;
      for (int r = 0; r < lim; r++) {
        uint32_t I = 0;
        for (int j = 0; j < (int)bl.size() && j < 6; j++) I |= (uint32_t)((r >> j) & 1) << bl[j];
        s.stab.push_back((int32_t)I);
      }
    }
  } else if (cell) {
    dg.variant = kVarCell;
    dg.rls = (uint8_t)cb;
    dg.sl = (uint8_t)std::max(0, G.L - 6);
    dg.lk = (uint8_t)(6 - std::min(G.L, 6));
    // operands by the first summed bit above the lanes they hold (the
    // serial cells are summed in that order, each operand multiplying
    // only the cells still open at its level): bit 6, then bit 7, then
    // none; without serial bits every operand is at the first level
    std::vector<int> lev(G.ops.size(), 0);
    for (size_t k = 0; k < G.ops.size(); k++) {
      const uint32_t m = G.ops[k].mask;
      lev[k] = G.L <= 6 ? 0 : ((m >> 6) & 1u) ? 0 : (G.L > 7 && ((m >> 7) & 1u)) ? 1 : 2;
      cls[k] = lev[k] < 2 ? kClsStep : kClsUnit;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return lev[a] < lev[b]; });
    int n0 = 0, n1 = 0;
    for (int k : order) {
      n0 += lev[k] == 0 ? 1 : 0;
      n1 += lev[k] == 1 ? 1 : 0;
    }
    dg.n_step = (uint8_t)n0;
    dg.n_serial = (uint8_t)n1;
    dg.n_units = 1u << (G.w - low - rb);
  } else if (stream) {
    dg.variant = kVarStream;
    dg.rls = (uint8_t)rls;
    dg.sl = (uint8_t)sl;
    dg.lk = (uint8_t)(6 - rls);
    // lane-kept bits: the lowest kept bits, so that the lanes' output
    // writes are contiguous (positions past the union, in narrow
    // groups, give idle lanes).  Choosing instead the bits the large
    // operands lack, so that lanes share operand elements, measured
    // slower.
    for (int j = 0; j < dg.lk; j++) dg.lkpos[j] = (uint8_t)(G.L + j);
    uint32_t lane_kept = 0;
    for (int j = 0; j < dg.lk; j++)
      if (dg.lkpos[j] < 32) lane_kept |= 1u << dg.lkpos[j];
    const uint32_t serial_bits = ((1u << G.L) - 1u) & ~((1u << (1 + rls)) - 1u);
    const uint32_t lane_bits = (((1u << rls) - 1u) << 1) | lane_kept;
    for (size_t k = 0; k < G.ops.size(); k++) {
      const Operand &o = G.ops[k];
      if (o.level >= 1 + rls)
        cls[k] = (o.mask & lane_bits) ? kClsSerial : kClsUniform;
      else
        cls[k] = (o.mask & serial_bits) ? kClsStep : kClsUnit;
    }
    // step-class operands with bit 0 first: they fill the unrolled slots
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      if (cls[a] != cls[b]) return cls[a] < cls[b];
      if (cls[a] == kClsStep) return (G.ops[a].mask & 1u) > (G.ops[b].mask & 1u);
      return false;
    });
    int nu = 0, ns = 0, nun = 0, nse = 0, ns0 = 0;
    for (int k : order) {
      if (cls[k] == kClsUnit) nu++;
      else if (cls[k] == kClsStep) {
        ns++;
        ns0 += (G.ops[k].mask & 1u) ? 1 : 0;
      }
      else if (cls[k] == kClsUniform) nun++;
      else nse++;
    }
    dg.n_unit = (uint8_t)nu;
    dg.n_step = (uint8_t)ns;
    dg.n_step0 = (uint8_t)ns0;
    dg.n_serial = (uint8_t)(nun + nse);
    dg.level_end[0] = (uint8_t)nun;
    const int kept_lanes = G.L + dg.lk;
    dg.n_units = G.w > kept_lanes ? 1u << (G.w - kept_lanes) : 1u;
  } else {
    dg.variant = kVarGeneric;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return G.ops[a].level < G.ops[b].level; });
    int cum = 0;
    for (int l = 0; l < kMaxLevels; l++) {
      if (l < G.L) cum += per_level[l];
      dg.level_end[l] = (uint8_t)cum;
    }
    const int bits = kGenRegBits + 6;
    dg.n_units = G.w > bits ? 1u << (G.w - bits) : 1u;
  }
  if (mfma) {
    // matrix form: m bits, then n bits, then batch bits
    uint8_t up[32];
    std::memset(up, 0, sizeof up);
    int j = 0;
    for (int q : gsh.mbits) up[j++] = (uint8_t)q;
    for (int q : gsh.nbits) up[j++] = (uint8_t)q;
    for (int q : gsh.bbits) up[j++] = (uint8_t)q;
    dg.n_ubits = 0;
    s.uperm.insert(s.uperm.end(), up, up + 32);
  } else {
    // wave-unit bits, those that large operands lack first (their data
    // is then reused by neighbouring units of the same block and XCD);
    // cells: the first rb of that order are the register bits (each
    // value of an operand lacking them serves several cells), first in
    // the table
    const int start = stream ? G.L : (cell ? low : kGenRegBits + 6);
    std::vector<std::pair<double, int>> sc;
    for (int b = start; b < G.w; b++) {
      bool lane = false;
      for (int j = 0; stream && j < dg.lk; j++) lane |= dg.lkpos[j] == b;
      if (lane) continue;
      double miss = 0;
      for (const Operand &o : G.ops)
        if (pl.tensors[o.tensor].gate < 0 && !((o.mask >> b) & 1u))
          miss += std::ldexp(1.0, (int)pl.tensors[o.tensor].vars.size());
      sc.push_back({-miss, b});
    }
    std::stable_sort(sc.begin(), sc.end());
    std::vector<int> regs;
    if (cell) {
      // register bits: one at a time, the kept bit that adds the fewest
      // loads (an operand is loaded once per distinct value of the cell
      // bits it holds), ties to the earlier bit of the order above
      // cell bits held so far: the serial bits still open at the
      // operand's level
      std::vector<uint32_t> held(G.ops.size(), 0);
      for (size_t k = 0; k < G.ops.size(); k++) {
        const uint32_t m = G.ops[k].mask;
        const int lv = G.L <= 6 ? 0 : ((m >> 6) & 1u) ? 0 : (G.L > 7 && ((m >> 7) & 1u)) ? 1 : 2;
        for (int t = lv; t < dg.sl; t++) held[k] += (m >> (6 + t)) & 1u;
      }
      for (int j = 0; j < rb; j++) {
        size_t bi = 0;
        double best_cost = -1;
        for (size_t q = 0; q < sc.size(); q++) {
          double cost = 0;
          for (size_t k = 0; k < G.ops.size(); k++)
            cost += std::ldexp(1.0, (int)held[k] + (int)((G.ops[k].mask >> sc[q].second) & 1u));
          if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            bi = q;
          }
        }
        for (size_t k = 0; k < G.ops.size(); k++) held[k] += (G.ops[k].mask >> sc[bi].second) & 1u;
        regs.push_back(sc[bi].second);
        sc.erase(sc.begin() + bi);
      }
      // with serial bits, the operands without them that hold no unit
      // bit go first: their product over the register cells is formed
      // once per angle set and reused by every unit (without serial
      // bits it would span every cell and cost more registers than it
      // saves)
      if (dg.sl > 0) {
        uint32_t unit_mask = 0;
        for (auto &q : sc) unit_mask |= 1u << q.second;
        const int last0 = dg.n_step + (dg.sl == 2 ? dg.n_serial : 0);
        std::stable_partition(order.begin() + last0, order.end(),
                              [&](int k) { return (G.ops[k].mask & unit_mask) == 0; });
        int nfix = 0;
        for (size_t i = last0; i < order.size(); i++)
          nfix += (G.ops[order[i]].mask & unit_mask) == 0 ? 1 : 0;
        dg.n_step0 = (uint8_t)nfix;
      } else {
        // without serial bits, the operands holding only lane bits go
        // first: their product, one value per lane, is formed once per
        // angle set and multiplies the cells once per unit
        std::stable_partition(order.begin(), order.end(),
                              [&](int k) { return (G.ops[k].mask & ~63u) == 0; });
        int nfix = 0;
        for (int k : order) nfix += (G.ops[k].mask & ~63u) == 0 ? 1 : 0;
        dg.n_step0 = (uint8_t)nfix;
      }
      // the cell mapping forms an operand's unit offset from its runs
      // over the unit bits; past kCellURuns of them, ascending order
      // (at most one run per two unit bits)
      int worst = 0;
      for (const Operand &o : G.ops) {
        int runs = 0, prev = -2;
        for (size_t j = 0; j < sc.size(); j++) {
          const int q = sc[j].second;
          if (!((o.mask >> q) & 1u)) {
            prev = -2;
            continue;
          }
          const int rank = __builtin_popcount(o.mask & ((1u << q) - 1u));
          if (rank != prev + 1) runs++;
          prev = rank;
        }
        worst = std::max(worst, runs);
      }
      if (worst > kCellURuns)
        std::sort(sc.begin(), sc.end(),
                  [](const std::pair<double, int> &a, const std::pair<double, int> &b) {
                    return a.second < b.second;
                  });
    }
    uint8_t up[32];
    std::memset(up, 0, sizeof up);
    const int first = cell ? rb : 0;
    for (int j = 0; j < first; j++) up[j] = (uint8_t)regs[j];
    for (size_t j = 0; j < sc.size(); j++) up[first + j] = (uint8_t)sc[j].second;
    dg.n_ubits = (uint8_t)sc.size();
    s.uperm.insert(s.uperm.end(), up, up + 32);
  }
  for (int k : order) {
    const Operand &o = G.ops[k];
    const Tensor &t = pl.tensors[o.tensor];
    DevOp d;
    std::memset(&d, 0, sizeof d);
    if (t.gate >= 0) {
      // gate operands read the table of the group's own precision
      d.off = env.table[G.prec] +
              gate_offset((*env.gates)[t.gate], t.transposed, env.p, env.slice) * es(G.prec);
      d.sstride = env.table_sstride[G.prec];
      d.dt = (uint8_t)G.prec;
    } else {
      d.off = env.arena + t.offset;
      d.sstride = env.arena_sstride;
      d.dt = (uint8_t)t.prec;
    }
    d.mask = o.mask;
    d.level = (uint8_t)o.level;
    uint8_t rs[32], rl[32], rd[32];
    const int nr = mask_runs(o.mask, rs, rl, rd);
    if (nr > kOpRuns) return set_err(QTN_ERANGE, "operand index set too fragmented");
    d.nruns = (uint8_t)nr;
    for (int r = 0; r < nr; r++)
      d.run[r] = (uint16_t)(rs[r] | (rl[r] << 5) | (rd[r] << 11));
    d.cls = (uint8_t)cls[k];
    d.stab = -1;
    if (stream && cls[k] != kClsUnit) {
      d.stab = (int32_t)s.stab.size();
      for (uint32_t st = 0; st < (1u << dg.sl); st++)
        s.stab.push_back((int32_t)pext32(st << (1 + dg.rls), o.mask));
    }
    if (cell) {
      // cell offsets (cell c: kept bits c % 2^rb, serial bits c / 2^rb),
      // then the runs giving the unit part of the index from the unit
      // number
      d.stab = (int32_t)s.stab.size();
      const uint8_t *rp = s.uperm.data() + s.uperm.size() - 32;
      uint32_t cm = 0;
      // serial cell bit rb + t is union bit 6 + sl - 1 - t (bit 6 the
      // highest cell bit, summed first)
      for (int j = 0; j < rb; j++) cm |= ((o.mask >> rp[j]) & 1u) << j;
      for (int t = 0; t < dg.sl; t++)
        cm |= ((o.mask >> (6 + dg.sl - 1 - t)) & 1u) << (rb + t);
      for (uint32_t c = 0; c < (1u << cb); c++) {
        uint32_t I = 0;
        for (int j = 0; j < rb; j++) I |= ((c >> j) & 1u) << rp[j];
        for (int t = 0; t < dg.sl; t++) I |= ((c >> (rb + t)) & 1u) << (6 + dg.sl - 1 - t);
        s.stab.push_back((int32_t)pext32(I, o.mask));
      }
      const uint8_t *up = rp + rb;
      uint16_t ur[kCellURuns];
      std::memset(ur, 0, sizeof ur);
      int nur = 0;
      for (int j = 0; j < dg.n_ubits;) {
        const int q = up[j];
        if (!((o.mask >> q) & 1u)) {
          j++;
          continue;
        }
        const int dst = __builtin_popcount(o.mask & ((1u << q) - 1u));
        int len = 1;
        while (j + len < dg.n_ubits && ((o.mask >> up[j + len]) & 1u) &&
               __builtin_popcount(o.mask & ((1u << up[j + len]) - 1u)) == dst + len)
          len++;
        if (nur == kCellURuns) return set_err(QTN_ERANGE, "cell mapping: unit runs");
        ur[nur++] = (uint16_t)(j | (len << 5) | (dst << 11));
        j += len;
      }
      dg.n_unit = (uint8_t)std::max<int>(dg.n_unit, nur);
      for (int w = 0; w < kCellURuns / 2; w++)
        s.stab.push_back((int32_t)((uint32_t)ur[2 * w] | ((uint32_t)ur[2 * w + 1] << 16)));
      s.stab.push_back((int32_t)cm);
    }
    if (mfma) {
      // the operand's element offsets of the tile's rows (side A) or
      // columns (side B), then of the summed indices
      d.stab = (int32_t)s.stab.size();
      const int sd = gsh.role[k];
      const int lim = sd == 0 ? kMmTM : kMmTN;
      const int32_t *rows = s.stab.data() + dg.gtab + (sd == 0 ? 0 : kMmTM);
      std::vector<int32_t> tab(lim + (1 << G.L));
      for (int r = 0; r < lim; r++) tab[r] = (int32_t)pext32((uint32_t)rows[r], o.mask);
      for (int kk = 0; kk < (1 << G.L); kk++) tab[lim + kk] = (int32_t)pext32((uint32_t)kk, o.mask);
      s.stab.insert(s.stab.end(), tab.begin(), tab.end());
    }
    if (d.dt != dg.prec) dg.cvt = 1;
    s.ops.push_back(d);
  }
  double gb = in_bytes + es(G.prec) * std::ldexp(1.0, G.w - G.L), gf = 0;
  for (int l = 0; l < G.L; l++) {
    int factors = per_level[l] + (l > 0 ? 1 : 0);
    gf += std::ldexp(1.0, G.w - l) * 6.0 * std::max(0, factors - 1) +
          std::ldexp(1.0, G.w - l - 1) * 2.0;
  }
  *dg_out = dg;
  *bytes_out = gb;
  *flops_out = gf;
  return QTN_OK;
}

// persistent: the schedule runs in a persistent executor (every group inside
// a workgroup, so no group takes the cell mapping).
int build_schedule(qtn_network *const *nets, int n, Schedule *S, const Force *force = nullptr,
                   int singleton_width = 0, int n_sets = 1, bool persistent = false) {
  Schedule &s = *S;
  s = Schedule();
  s.serial = ++g_sched_serial;
  s.n_sets = n_sets;
  s.prec = nets[0]->precision;
  s.scalar_prec = s.prec == kPrecC64 ? 1 : 0;
  auto al = [](int64_t bytes) { return (bytes + 255) / 256 * 256; };
  auto es = [](int prec) { return prec == 1 ? (int64_t)8 : (int64_t)16; };
  // every offset below is in bytes from the data base
  int64_t data = 0;
  int n_scalars = 0;
  for (int i = 0; i < n; i++) {
    if (nets[i]->precision != s.prec) return set_err(QTN_EINVAL, "batched networks differ in precision");
    // one copy of every table, scalar slot and arena per angle set
    FillDesc f{(int64_t)s.n_angles, -1, -1, 0, 0, nets[i]->p, 0};
    const int64_t tab = gate_table_elems(nets[i]->p);
    if (s.prec != kPrecC64) {
      f.table128 = data;
      f.sstride128 = al(tab * 16);
      data += n_sets * f.sstride128;
    }
    if (s.prec != kPrecC128) {
      f.table64 = data;
      f.sstride64 = al(tab * 8);
      data += n_sets * f.sstride64;
    }
    s.fills.push_back(f);
    s.n_angles += 2 * nets[i]->p;
    for (auto &pl : nets[i]->plans) n_scalars += pl.n_scalars * pl.n_slices;
  }
  s.scalar_off = data;
  s.scalar_sstride = al(n_scalars * es(s.scalar_prec));
  data += n_sets * s.scalar_sstride;
  int scalar_next = 0;
  s.ncb.push_back(0);
  for (int i = 0; i < n; i++) {
    const qtn_network *net = nets[i];
    const int64_t table[2] = {s.fills[i].table128, s.fills[i].table64};
    const int64_t table_sstride[2] = {s.fills[i].sstride128, s.fills[i].sstride64};
    for (size_t c = 0; c < net->plans.size(); c++) {
      const ConePlan &pl = net->plans[c];
      const std::vector<Gate> &gates = pl.gates.empty() ? net->cones[c].gates : pl.gates;
      const int64_t arena = data, arena_sstride = al(pl.arena_bytes);
      data += n_sets * arena_sstride;
      s.csb.push_back(scalar_next);
      s.cns.push_back(pl.n_slices);
      // hybrid executor (executor 5): a cone with a bucket wider than the
      // network's hybrid width runs by per-group launches
      const bool heavy = persistent && net->executor == 5 && pl.max_width > net->hybrid_width;
      s.cone_heavy.push_back(heavy ? 1 : 0);
      std::vector<Task> tasks;
      int open_begin = -1;
      double seg_bytes = 0, seg_flops = 0;
      auto close_segment = [&](int end) {
        if (open_begin < 0) return;
        s.ranges.push_back(make_int2(open_begin, end));
        tasks.push_back({QTN_K_BLOCK, (int)s.ranges.size() - 1, 0, 0, seg_bytes, seg_flops});
        open_begin = -1;
        seg_bytes = seg_flops = 0;
      };
      // index slicing: the groups run once per slice, in order, on the one
      // arena; slice k's scalars take slots k * n_scalars onwards
      for (int slice = 0; slice < pl.n_slices; slice++)
      for (const Group &G : pl.groups) {
        if (G.ops.size() > 255) return set_err(QTN_ERANGE, "bucket with more than 255 tensors");
        if (G.out_tensor < 0 && G.prec != s.scalar_prec)
          return set_err(QTN_EINVAL, "scalar group precision differs from the scalar slots");
        GroupEnv env;
        env.out_off = G.out_tensor >= 0
                          ? arena + pl.tensors[G.out_tensor].offset
                          : s.scalar_off + (int64_t)(scalar_next + slice * pl.n_scalars + G.scalar_slot) *
                                               es(s.scalar_prec);
        env.out_sstride = G.out_tensor >= 0 ? arena_sstride : s.scalar_sstride;
        env.arena = arena;
        env.arena_sstride = arena_sstride;
        for (int q = 0; q < 2; q++) {
          env.table[q] = table[q];
          env.table_sstride[q] = table_sstride[q];
        }
        env.gates = &gates;
        env.slice = (uint32_t)slice;
        env.p = net->p;
        // the mapping requested (network config, tuned pick or a tuning
        // candidate); 0 leaves it to the width rule
        env.var_req = net->variant;
        env.rls_req = net->lane_sum_bits;
        if (G.pick_variant > 0) {
          env.var_req = G.pick_variant;
          if (G.pick_rls >= 0) env.rls_req = G.pick_rls;
        }
        const bool is_small = force && force->place >= 0
                                  ? force->place == 0
                                  : (G.pick_place >= 0 ? G.pick_place == 0 : G.small);
        if (force) {
          env.var_req = force->variant;
          env.rls_req = force->rls;
        }
        env.is_small = is_small;
        env.persistent = persistent && !heavy;
        DevGroup dg;
        double gb = 0, gf = 0;
        const int rc = describe_group(G, pl, env, s, &dg, &gb, &gf);
        if (rc) return rc;
        const int gid = (int)s.groups.size();
        s.groups.push_back(dg);
        s.group_cone.push_back(s.n_cones);
        s.group_index.push_back((int)(&G - pl.groups.data()));
        if (singleton_width > 0 && G.w <= singleton_width) s.singles.push_back(gid);
        if (is_small) {
          if (open_begin < 0) open_begin = gid;
          seg_bytes += gb;
          seg_flops += gf;
        } else {
          close_segment(gid);
          tasks.push_back({QTN_K_WIDE, gid, dg.n_units, dg.variant, gb, gf});
        }
      }
      close_segment((int)s.groups.size());
      scalar_next += pl.n_scalars * pl.n_slices;
      s.cone_tasks.push_back(std::move(tasks));
      s.n_cones++;
    }
    s.ncb.push_back(s.n_cones);
  }
  s.csb.push_back(scalar_next);
  // the first n_cones ranges are the leading small segments (possibly empty)
  std::vector<int2> lead(s.n_cones, make_int2(0, 0));
  for (int c = 0; c < s.n_cones; c++) {
    auto &tk = s.cone_tasks[c];
    if (!tk.empty() && tk[0].kind == QTN_K_BLOCK) {
      lead[c] = s.ranges[tk[0].index];
      s.init_bytes += tk[0].bytes;
      s.init_flops += tk[0].flops;
      tk.erase(tk.begin());
    }
  }
  for (auto &tk : s.cone_tasks)
    for (auto &t : tk)
      if (t.kind == QTN_K_BLOCK) t.index += s.n_cones;
  s.ranges.insert(s.ranges.begin(), lead.begin(), lead.end());
  s.singles_range0 = (int)s.ranges.size();
  for (int g : s.singles) s.ranges.push_back(make_int2(g, g + 1));
  s.n_nets = n;
  // persistent work items: the j-th task of every cone forms step j (leading
  // segment first); inside a step the costlier cones come first.  The
  // lockstep executor runs the steps between grid barriers; the dataflow
  // executor takes items in the same order and waits only for the previous
  // task of the item's own cone.
  {
    std::vector<int> corder(s.n_cones);
    std::vector<double> ccost(s.n_cones, 0);
    for (int c = 0; c < s.n_cones; c++) {
      corder[c] = c;
      for (auto &t : s.cone_tasks[c]) ccost[c] += t.bytes;
    }
    std::stable_sort(corder.begin(), corder.end(), [&](int a, int b) { return ccost[a] > ccost[b]; });
    std::vector<std::vector<int4>> per_step;
    std::vector<std::vector<int>> per_step_task;
    for (int cn : corder) {
      // a heavy cone runs by launches after the persistent kernel; its
      // leading segment, which needs nothing, is a first-step item
      const bool heavy = s.cone_heavy[cn] != 0;
      int j = 0, prev = -1;
      auto put = [&](const int4 &it, int task) {
        if ((int)per_step.size() <= j) {
          per_step.resize(j + 1);
          per_step_task.resize(j + 1);
        }
        per_step[j].push_back(it);
        per_step_task[j].push_back(task);
      };
      auto new_task = [&]() {
        s.task_dep.push_back(prev);
        s.task_need.push_back(0);
        prev = (int)s.task_dep.size() - 1;
        return prev;
      };
      if (lead[cn].y > lead[cn].x) {
        const int tk = new_task();
        put(make_int4(lead[cn].x, lead[cn].y, 0, 0), tk);
        s.task_need[tk]++;
        j++;
      }
      if (heavy) continue;
      for (const Task &t : s.cone_tasks[cn]) {
        const int tk = new_task();
        if (t.kind == QTN_K_BLOCK) {
          const int2 r = s.ranges[t.index];
          put(make_int4(r.x, r.y, 0, 0), tk);
          s.task_need[tk]++;
        } else {
          const uint32_t nu = t.n_units;
          // at least four passes of the block's waves per item
          uint32_t chunk = std::max<uint32_t>(16u, nu / 1024u);
          for (uint32_t u = 0; u < nu; u += chunk) {
            put(make_int4(t.index, -1, (int)u, (int)std::min(nu, u + chunk)), tk);
            s.task_need[tk]++;
          }
        }
        j++;
      }
    }
    s.step_begin.push_back(0);
    for (size_t j = 0; j < per_step.size(); j++) {
      s.items.insert(s.items.end(), per_step[j].begin(), per_step[j].end());
      s.item_task.insert(s.item_task.end(), per_step_task[j].begin(), per_step_task[j].end());
      s.step_begin.push_back((int)s.items.size());
    }
    s.n_steps = (int)per_step.size();
    s.n_tasks = (int)s.task_dep.size();
    s.n_ctl = 4 + std::max(s.n_steps, s.n_tasks);
    // ready-queue tables: a task's items are contiguous (one cone's chunks of
    // one step); the first step holds the first task of every cone
    s.task_next.assign(s.n_tasks, -1);
    for (int t = 1; t < s.n_tasks; t++)
      if (s.task_dep[t] >= 0) s.task_next[s.task_dep[t]] = t;
    s.task_first.assign(s.n_tasks, -1);
    for (int i = (int)s.item_task.size() - 1; i >= 0; i--) s.task_first[s.item_task[i]] = i;
    s.n_init = s.n_steps > 0 ? s.step_begin[1] : 0;
  }
  s.bytes[QTN_K_BLOCK] = s.init_bytes;
  s.flops[QTN_K_BLOCK] = s.init_flops;
  // a wide launch walks the units of every set in one flat 31-bit index
  for (const DevGroup &g : s.groups)
    if ((uint64_t)g.n_units * (uint64_t)s.n_sets > 0x7FFFFFFFull)
      return set_err(QTN_ERANGE, "too many units over the angle sets for one launch");
  for (auto &tk : s.cone_tasks)
    for (auto &t : tk) {
      s.bytes[t.kind] += t.bytes;
      s.flops[t.kind] += t.flops;
    }

  // workspace layout (bytes)
  s.off_res = 0;
  s.off_angles = align_up(8 * (size_t)(2 * s.n_cones + s.n_nets) * s.n_sets, 256);
  s.off_desc = align_up(s.off_angles + 8 * (size_t)s.n_angles * s.n_sets, 256);
  s.off_fills = s.off_desc;
  s.off_groups = align_up(s.off_fills + sizeof(FillDesc) * s.fills.size(), 256);
  s.off_ops = align_up(s.off_groups + sizeof(DevGroup) * s.groups.size(), 256);
  s.off_stab = align_up(s.off_ops + sizeof(DevOp) * s.ops.size(), 256);
  s.off_uperm = align_up(s.off_stab + sizeof(int32_t) * s.stab.size(), 256);
  s.off_ranges = align_up(s.off_uperm + s.uperm.size(), 256);
  s.off_csb = align_up(s.off_ranges + sizeof(int2) * s.ranges.size(), 256);
  s.off_ncb = align_up(s.off_csb + sizeof(int) * s.csb.size(), 256);
  s.off_cns = align_up(s.off_ncb + sizeof(int) * s.ncb.size(), 256);
  s.off_items = align_up(s.off_cns + sizeof(int) * s.cns.size(), 256);
  s.off_steps = align_up(s.off_items + sizeof(int4) * s.items.size(), 256);
  s.off_item_task = align_up(s.off_steps + sizeof(int) * s.step_begin.size(), 256);
  s.off_task_next = align_up(s.off_item_task + sizeof(int) * s.item_task.size(), 256);
  s.off_task_first = align_up(s.off_task_next + sizeof(int) * s.task_next.size(), 256);
  s.off_task_need = align_up(s.off_task_first + sizeof(int) * s.task_first.size(), 256);
  s.off_queue = align_up(s.off_task_need + sizeof(int) * s.task_need.size(), 256);
  s.off_ctl = align_up(s.off_queue + sizeof(uint32_t) * s.items.size(), 256);
  s.off_data = align_up(s.off_ctl + sizeof(uint32_t) * s.n_ctl, 256);
  s.total = s.off_data + (size_t)data;
  s.desc_blob.assign(s.off_data - s.off_desc, 0);
  auto put = [&](size_t off, const void *src, size_t bytes) {
    if (bytes) std::memcpy(s.desc_blob.data() + (off - s.off_desc), src, bytes);
  };
  put(s.off_fills, s.fills.data(), sizeof(FillDesc) * s.fills.size());
  put(s.off_groups, s.groups.data(), sizeof(DevGroup) * s.groups.size());
  put(s.off_ops, s.ops.data(), sizeof(DevOp) * s.ops.size());
  put(s.off_stab, s.stab.data(), sizeof(int32_t) * s.stab.size());
  put(s.off_uperm, s.uperm.data(), s.uperm.size());
  put(s.off_ranges, s.ranges.data(), sizeof(int2) * s.ranges.size());
  put(s.off_csb, s.csb.data(), sizeof(int) * s.csb.size());
  put(s.off_ncb, s.ncb.data(), sizeof(int) * s.ncb.size());
  put(s.off_cns, s.cns.data(), sizeof(int) * s.cns.size());
  put(s.off_items, s.items.data(), sizeof(int4) * s.items.size());
  put(s.off_steps, s.step_begin.data(), sizeof(int) * s.step_begin.size());
  put(s.off_item_task, s.item_task.data(), sizeof(int) * s.item_task.size());
  put(s.off_task_next, s.task_next.data(), sizeof(int) * s.task_next.size());
  put(s.off_task_first, s.task_first.data(), sizeof(int) * s.task_first.size());
  put(s.off_task_need, s.task_need.data(), sizeof(int) * s.task_need.size());
  return QTN_OK;
}

int ensure_runtime(Runtime &rt, int n_streams, int n_res) {
  int dev = 0;
  QTN_HIP(hipGetDevice(&dev));
  if (rt.device >= 0 && rt.device != dev) rt.release();
  if (rt.device < 0) {
    rt.device = dev;
    QTN_HIP(hipStreamCreateWithFlags(&rt.main, hipStreamNonBlocking));
    for (int i = 0; i < n_streams; i++) {
      hipStream_t s;
      QTN_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      rt.side.push_back(s);
      hipEvent_t e;
      QTN_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      rt.ev_join.push_back(e);
    }
    QTN_HIP(hipEventCreateWithFlags(&rt.ev_in, hipEventDisableTiming));
    QTN_HIP(hipEventCreateWithFlags(&rt.ev_fork, hipEventDisableTiming));
    QTN_HIP(hipHostMalloc((void **)&rt.pinned_err, 4 * sizeof(uint32_t), hipHostMallocDefault));
    int n_cu = 0;
    QTN_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    rt.persist_blocks = persistent_blocks(kPrecC128, n_cu);
  }
  // a runtime first made for a one-stream pass (autotuning) grows to the
  // network's stream count
  while ((int)rt.side.size() < n_streams) {
    hipStream_t s;
    QTN_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    rt.side.push_back(s);
    hipEvent_t e;
    QTN_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    rt.ev_join.push_back(e);
  }
  if (rt.pinned_n < (size_t)n_res) {
    if (rt.pinned) QTN_HIP(hipHostFree(rt.pinned));
    rt.pinned = nullptr;
    QTN_HIP(hipHostMalloc((void **)&rt.pinned, sizeof(double) * n_res, hipHostMallocDefault));
    rt.pinned_n = n_res;
  }
  return QTN_OK;
}

struct Timer {
  bool on = false;
  struct Rec {
    int kind;
    hipEvent_t a, b;
    int group, n_groups;
    double bytes, flops;
  };
  std::vector<Rec> recs;
  // on_dispatch: the launch attaches the events to its kernel's dispatch
  // (t0(), t1()) instead of recording them around it on the stream
  int begin(int kind, hipStream_t s, int group = -1, int n_groups = 0, double bytes = 0,
            double flops = 0, bool on_dispatch = false) {
    if (!on) return QTN_OK;
    Rec r{kind, nullptr, nullptr, group, n_groups, bytes, flops};
    QTN_HIP(hipEventCreate(&r.a));
    QTN_HIP(hipEventCreate(&r.b));
    if (!on_dispatch) QTN_HIP(hipEventRecord(r.a, s));
    recs.push_back(r);
    return QTN_OK;
  }
  hipEvent_t t0() const { return on ? recs.back().a : nullptr; }
  hipEvent_t t1() const { return on ? recs.back().b : nullptr; }
  int end(hipStream_t s, bool on_dispatch = false) {
    if (!on || on_dispatch) return QTN_OK;
    QTN_HIP(hipEventRecord(recs.back().b, s));
    return QTN_OK;
  }
  ~Timer() {
    for (auto &r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
  }
};

// Blocks of the persistent launch: all that are resident at once, or the
// tuned share of them (whole rounds over the 8 XCDs, at least 8).
int persist_grid(const Exec &X) {
  const int full = X.rt.persist_blocks;
  if (X.grid_quarters >= 4 || full <= 8) return full;
  const int nb = full * X.grid_quarters / 4;
  return std::max(8, nb - nb % 8);
}

// Orders the items inside every lockstep step: 0 the costliest light cone's
// first (as built), 1 reversed.  The blob's copies are rewritten and the
// schedule takes a new serial, so the next run uploads them.
void set_item_order(Schedule &s, int order) {
  if (order == s.item_order) return;
  for (int j = 0; j < s.n_steps; j++) {
    std::reverse(s.items.begin() + s.step_begin[j], s.items.begin() + s.step_begin[j + 1]);
    std::reverse(s.item_task.begin() + s.step_begin[j],
                 s.item_task.begin() + s.step_begin[j + 1]);
  }
  if (!s.items.empty())
    std::memcpy(s.desc_blob.data() + (s.off_items - s.off_desc), s.items.data(),
                sizeof(int4) * s.items.size());
  if (!s.item_task.empty())
    std::memcpy(s.desc_blob.data() + (s.off_item_task - s.off_desc), s.item_task.data(),
                sizeof(int) * s.item_task.size());
  s.item_order = order;
  s.serial = ++g_sched_serial;
}

void drop_graph(Runtime &rt) {
  if (rt.exec) (void)hipGraphExecDestroy(rt.exec);
  if (rt.graph) (void)hipGraphDestroy(rt.graph);
  rt.exec = nullptr;
  rt.graph = nullptr;
}

// Every launch of one evaluation, on rt.main and the side streams.
int enqueue(Exec &X, Timer &tm) {
  Schedule &s = X.sched;
  Runtime &rt = X.rt;
  char *ws = (char *)rt.ws;
  void *data = ws + s.off_data;
  auto *groups = (const DevGroup *)(ws + s.off_groups);
  auto *ops = (const DevOp *)(ws + s.off_ops);
  auto *ranges = (const int2 *)(ws + s.off_ranges);
  auto *stab = (const int32_t *)(ws + s.off_stab);
  auto *uperm = (const uint8_t *)(ws + s.off_uperm);
  int rc;
  if ((rc = tm.begin(QTN_K_FILL, rt.main))) return rc;
  QTN_HIP(launch_fill(s.prec, data, (const double *)(ws + s.off_angles),
                      (const FillDesc *)(ws + s.off_fills), s.n_nets, s.n_angles, s.n_sets,
                      rt.main));
  if ((rc = tm.end(rt.main))) return rc;
  const int NS = s.n_sets;  // launch records carry the bytes of every set
  if (X.persistent) {
    if (NS != 1) return set_err(QTN_EINVAL, "the persistent executors run one angle set");
    bool any_heavy = false;
    for (char h : s.cone_heavy) any_heavy |= h != 0;
    // the persistent launch runs alone: its grid barriers need every block
    // resident, which kernels running beside it could prevent (measured: with
    // the heavy cones' launches started beside a full-size persistent grid, a
    // barrier wait ran past its bound)
    const int nb = persist_grid(X);
    if (nb < 1) return set_err(QTN_EDEVICE, "persistent kernel does not fit on the device");
    double b_all = 0, f_all = 0;
    for (int k = 0; k < QTN_NKERNELS; k++) {
      b_all += s.bytes[k];
      f_all += s.flops[k];
    }
    const int K = tm.on ? 1 : (int)rt.side.size();
    if (X.hybrid && any_heavy) {
      // the heavy cones' share is not the persistent launch's
      for (int c = 0; c < s.n_cones; c++)
        if (s.cone_heavy[c]) {
          for (auto &t : s.cone_tasks[c]) {
            b_all -= t.bytes;
            f_all -= t.flops;
          }
        }
    }
    if ((rc = tm.begin(QTN_K_PERSISTENT, rt.main, 0, (int)s.groups.size(), b_all, f_all, true)))
      return rc;
    if (X.dataflow)
      QTN_HIP(launch_dataflow(data, groups, ops, stab, uperm, (const int4 *)(ws + s.off_items),
                              (int)s.items.size(), s.n_init, (const int *)(ws + s.off_item_task),
                              (const int *)(ws + s.off_task_next),
                              (const int *)(ws + s.off_task_first),
                              (const int *)(ws + s.off_task_need), (uint32_t *)(ws + s.off_queue),
                              (uint32_t *)(ws + s.off_ctl), s.n_ctl, nb, X.spin_limit, rt.main,
                              tm.t0(), tm.t1()));
    else
      QTN_HIP(launch_persistent(s.prec, data, groups, ops, stab, uperm,
                                (const int4 *)(ws + s.off_items), (const int *)(ws + s.off_steps),
                                s.n_steps, (uint32_t *)(ws + s.off_ctl), s.n_ctl, nb, X.spin_limit,
                                rt.main, tm.t0(), tm.t1()));
    if ((rc = tm.end(rt.main, true))) return rc;
    if (X.hybrid && any_heavy) {
      // after the persistent launch (which ran their leading segments): the
      // heavy cones, each cone's tasks in order on one side stream, heaviest
      // first, dealt to the least loaded stream
      QTN_HIP(hipEventRecord(rt.ev_fork, rt.main));
      for (int i = 0; i < K; i++) QTN_HIP(hipStreamWaitEvent(rt.side[i], rt.ev_fork, 0));
      std::vector<int> order;
      std::vector<double> cost(s.n_cones, 0);
      for (int c = 0; c < s.n_cones; c++)
        if (s.cone_heavy[c]) {
          order.push_back(c);
          for (auto &t : s.cone_tasks[c]) cost[c] += t.bytes;
        }
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
      std::vector<double> load(K, 0);
      for (int c : order) {
        const int st = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[st] += cost[c];
        hipStream_t hs = rt.side[st];
        for (auto &t : s.cone_tasks[c]) {
          const int g0 = t.kind == QTN_K_BLOCK ? s.ranges[t.index].x : t.index;
          const int ng = t.kind == QTN_K_BLOCK ? s.ranges[t.index].y - s.ranges[t.index].x : 1;
          if ((rc = tm.begin(t.kind, hs, g0, ng, t.bytes, t.flops, true))) return rc;
          if (t.kind == QTN_K_BLOCK)
            QTN_HIP(launch_block_groups(s.prec, data, groups, ops, stab, uperm, ranges, t.index, 1,
                                        NS, hs, tm.t0(), tm.t1()));
          else
            QTN_HIP(launch_wide_group(s.groups[t.index], data, groups, ops, stab, uperm, t.index,
                                      NS, hs, tm.t0(), tm.t1()));
          if ((rc = tm.end(hs, true))) return rc;
        }
      }
      for (int i = 0; i < K; i++) {
        QTN_HIP(hipEventRecord(rt.ev_join[i], rt.side[i]));
        QTN_HIP(hipStreamWaitEvent(rt.main, rt.ev_join[i], 0));
      }
    }
  } else {
  // leading small segments: one launch for every cone before the fork, or
  // (lead_per_cone) each cone's own one-block launch on its stream
  if (!X.lead_per_cone) {
    if ((rc = tm.begin(QTN_K_BLOCK, rt.main, 0, (int)s.groups.size(), NS * s.init_bytes,
                       NS * s.init_flops, true)))
      return rc;
    QTN_HIP(launch_block_groups(s.prec, data, groups, ops, stab, uperm, ranges, 0, s.n_cones, NS,
                                rt.main, tm.t0(), tm.t1()));
    if ((rc = tm.end(rt.main, true))) return rc;
  }
  // timed runs serialize on one stream, so each event pair brackets one kernel
  const int K = tm.on ? 1 : (int)rt.side.size();
  bool any = X.lead_per_cone;
  for (auto &tk : s.cone_tasks) any |= !tk.empty();
  if (any) {
    QTN_HIP(hipEventRecord(rt.ev_fork, rt.main));
    for (int i = 0; i < K; i++) QTN_HIP(hipStreamWaitEvent(rt.side[i], rt.ev_fork, 0));
    // heaviest light cones first, dealt round-robin over the side streams
    std::vector<int> order(s.n_cones);
    std::vector<double> cost(s.n_cones, 0);
    for (int c = 0; c < s.n_cones; c++) {
      order[c] = c;
      for (auto &t : s.cone_tasks[c]) cost[c] += t.bytes;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<double> load(K, 0);
    for (int c : order) {
      const bool lead = X.lead_per_cone && s.ranges[c].y > s.ranges[c].x;
      if (s.cone_tasks[c].empty() && !lead) continue;
      int st = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[st] += cost[c];
      hipStream_t hs = rt.side[st];
      if (lead) {
        if ((rc = tm.begin(QTN_K_BLOCK, hs, s.ranges[c].x, s.ranges[c].y - s.ranges[c].x, 0, 0,
                           true)))
          return rc;
        QTN_HIP(launch_block_groups(s.prec, data, groups, ops, stab, uperm, ranges, c, 1, NS, hs,
                                    tm.t0(), tm.t1()));
        if ((rc = tm.end(hs, true))) return rc;
      }
      for (auto &t : s.cone_tasks[c]) {
        const int g0 = t.kind == QTN_K_BLOCK ? s.ranges[t.index].x : t.index;
        const int ng = t.kind == QTN_K_BLOCK ? s.ranges[t.index].y - s.ranges[t.index].x : 1;
        if ((rc = tm.begin(t.kind, hs, g0, ng, NS * t.bytes, NS * t.flops, true))) return rc;
        if (t.kind == QTN_K_BLOCK)
          QTN_HIP(launch_block_groups(s.prec, data, groups, ops, stab, uperm, ranges, t.index, 1, NS,
                                      hs, tm.t0(), tm.t1()));
        else
          QTN_HIP(launch_wide_group(s.groups[t.index], data, groups, ops, stab, uperm, t.index, NS,
                                    hs, tm.t0(), tm.t1()));
        if ((rc = tm.end(hs, true))) return rc;
      }
    }
    for (int i = 0; i < K; i++) {
      QTN_HIP(hipEventRecord(rt.ev_join[i], rt.side[i]));
      QTN_HIP(hipStreamWaitEvent(rt.main, rt.ev_join[i], 0));
    }
  }
  }
  if ((rc = tm.begin(QTN_K_REDUCE, rt.main))) return rc;
  QTN_HIP(launch_reduce(s.scalar_prec == 1 ? kPrecC64 : kPrecC128, data, s.scalar_off,
                        s.scalar_sstride, (const int *)(ws + s.off_csb),
                        (const int *)(ws + s.off_ncb), (const int *)(ws + s.off_cns), s.n_cones,
                        s.n_nets, NS,
                        (double *)(ws + s.off_res), rt.main));
  if ((rc = tm.end(rt.main))) return rc;
  return QTN_OK;
}

// Upload descriptors and angles, run, read back.  The descriptors go up
// before every evaluation: between calls the workspace belongs to the caller,
// who may reuse it for other schedules or other data.
// set_angles: n_sets * n_angles doubles (per set, per network gamma[p] then
// beta[p]); NULL: the networks' own angles (one set).
int run_exec(Exec &X, const std::vector<const qtn_network *> &nets, void *ws, size_t bytes,
             void *stream, int n_streams, bool eager, Timer &tm, std::vector<double> &res,
             const double *set_angles = nullptr) {
  Schedule &s = X.sched;
  Runtime &rt = X.rt;
  if (!ws) return set_err(QTN_EINVAL, "workspace is NULL");
  if (bytes < s.total)
    return set_err(QTN_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes, plan needs " +
                                   std::to_string(s.total));
  if ((uintptr_t)ws % 256) return set_err(QTN_EINVAL, "workspace must be 256-byte aligned");
  if (!set_angles && s.n_sets != 1) return set_err(QTN_EINVAL, "angle sets missing");
  const int n_res = (2 * s.n_cones + s.n_nets) * s.n_sets;
  int rc = ensure_runtime(rt, n_streams, std::max(n_res, s.n_angles * s.n_sets));
  if (rc) return rc;
  if (rt.desc_serial != s.serial || rt.pinned_desc_n != s.desc_blob.size()) {
    if (rt.pinned_desc_cap < s.desc_blob.size()) {
      if (rt.pinned_desc) QTN_HIP(hipHostFree(rt.pinned_desc));
      rt.pinned_desc = nullptr;
      rt.pinned_desc_cap = 0;
      QTN_HIP(hipHostMalloc((void **)&rt.pinned_desc, s.desc_blob.size(), hipHostMallocDefault));
      rt.pinned_desc_cap = s.desc_blob.size();
    }
    std::memcpy(rt.pinned_desc, s.desc_blob.data(), s.desc_blob.size());
    rt.pinned_desc_n = s.desc_blob.size();
    rt.desc_serial = s.serial;
  }
  QTN_HIP(hipEventRecord(rt.ev_in, (hipStream_t)stream));
  QTN_HIP(hipStreamWaitEvent(rt.main, rt.ev_in, 0));
  // the captured graph holds the old workspace's addresses
  if (rt.ws != ws) drop_graph(rt);
  rt.ws = ws;
  QTN_HIP(hipMemcpyAsync((char *)ws + s.off_desc, rt.pinned_desc, rt.pinned_desc_n,
                         hipMemcpyHostToDevice, rt.main));
  if (set_angles) {
    std::memcpy(rt.pinned, set_angles, sizeof(double) * s.n_angles * s.n_sets);
  } else {
    size_t a = 0;
    for (auto *net : nets) {
      for (int l = 0; l < net->p; l++) rt.pinned[a + l] = net->gamma[l];
      for (int l = 0; l < net->p; l++) rt.pinned[a + net->p + l] = net->beta[l];
      a += 2 * net->p;
    }
  }
  QTN_HIP(hipMemcpyAsync((char *)ws + s.off_angles, rt.pinned,
                         sizeof(double) * s.n_angles * s.n_sets, hipMemcpyHostToDevice, rt.main));
  if (eager || tm.on) {
    if ((rc = enqueue(X, tm))) return rc;
  } else {
    if (!rt.exec) {
      QTN_HIP(hipStreamBeginCapture(rt.main, hipStreamCaptureModeThreadLocal));
      rc = enqueue(X, tm);
      hipGraph_t graph = nullptr;
      hipError_t ce = hipStreamEndCapture(rt.main, &graph);
      if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (ce != hipSuccess)
        return set_err(QTN_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
      rt.graph = graph;
      QTN_HIP(hipGraphInstantiate(&rt.exec, rt.graph, nullptr, nullptr, 0));
    }
    QTN_HIP(hipGraphLaunch(rt.exec, rt.main));
  }
  QTN_HIP(hipMemcpyAsync(rt.pinned, (char *)ws + s.off_res, sizeof(double) * n_res,
                         hipMemcpyDeviceToHost, rt.main));
  if (X.persistent)
    QTN_HIP(hipMemcpyAsync(rt.pinned_err, (char *)ws + s.off_ctl, 4 * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, rt.main));
  QTN_HIP(hipStreamSynchronize(rt.main));
  if (X.persistent && rt.pinned_err[2] != 0)
    return set_err(QTN_EDEVICE, X.dataflow
                                    ? "persistent executor: a dependency wait exceeded its bound"
                                    : "persistent executor: a grid barrier wait exceeded its bound");
  res.assign(rt.pinned, rt.pinned + n_res);
  return QTN_OK;
}

bool finite_angles(int p, const double *g, const double *b) {
  for (int l = 0; l < p; l++)
    if (!std::isfinite(g[l]) || !std::isfinite(b[l])) return false;
  return true;
}

}  // namespace

extern "C" {

const char *qtn_last_error(void) { return g_err.c_str(); }

int qtn_network_build(int32_t n_vertices, int64_t n_edges, const int32_t *edges, int32_t p,
                      const double *gamma, const double *beta, const qtn_config *cfg,
                      qtn_network **out) {
  try {
    if (!out) return set_err(QTN_EINVAL, "out is NULL");
    if (p < 1 || p > 64) return set_err(QTN_EINVAL, "p must be in 1..64");
    if (!gamma || !beta) return set_err(QTN_EINVAL, "angles are NULL");
    if (!finite_angles(p, gamma, beta)) return set_err(QTN_EINVAL, "angles must be finite");
    std::unique_ptr<qtn_network> net(new qtn_network());
    std::string err = make_graph(n_vertices, n_edges, edges, &net->g);
    if (!err.empty()) return set_err(QTN_EINVAL, err);
    net->p = p;
    net->gamma.assign(gamma, gamma + p);
    net->beta.assign(beta, beta + p);
    if (cfg) {
      if (cfg->max_levels < 0 || cfg->max_levels > kMaxLevels)
        return set_err(QTN_EINVAL, "max_levels must be in 0..8");
      if (cfg->max_levels) net->opt.max_levels = cfg->max_levels;
      if (cfg->small_width < 0 || cfg->small_width > kMaxWidth)
        return set_err(QTN_EINVAL, "small_width must be in 0..32");
      if (cfg->small_width) net->opt.small_width = cfg->small_width;
      if (cfg->max_width < 0 || cfg->max_width > kMaxWidth)
        return set_err(QTN_EINVAL, "max_width must be in 0..32");
      if (cfg->max_width) net->opt.max_width = cfg->max_width;
      if (cfg->n_streams < 0 || cfg->n_streams > 16)
        return set_err(QTN_EINVAL, "n_streams must be in 0..16");
      if (cfg->n_streams) net->n_streams = cfg->n_streams;
      net->eager = cfg->eager != 0;
      if (cfg->lane_sum_bits < 0 || cfg->lane_sum_bits > 5)
        return set_err(QTN_EINVAL, "lane_sum_bits must be in 0..5");
      if (cfg->lane_sum_bits) net->lane_sum_bits = cfg->lane_sum_bits;
      if (cfg->variant < 0 || cfg->variant > 4) return set_err(QTN_EINVAL, "variant must be 0..4");
      net->variant = cfg->variant;
      if (cfg->order_trials < 0 || cfg->order_trials > 4096)
        return set_err(QTN_EINVAL, "order_trials must be in 0..4096");
      net->order_trials = cfg->order_trials;
      if (cfg->executor < 0 || cfg->executor > 5) return set_err(QTN_EINVAL, "executor must be 0..5");
      net->executor = cfg->executor;
      if (cfg->spin_limit > 0) net->spin_limit = (uint32_t)cfg->spin_limit;
      if (cfg->mixed_width < 0 || cfg->mixed_width > 32)
        return set_err(QTN_EINVAL, "mixed_width must be in 0..32");
      if (cfg->mixed_width > 0) net->opt.mixed_width = cfg->mixed_width;
      if (cfg->slice_width < 0 || cfg->slice_width > kMaxWidth)
        return set_err(QTN_EINVAL, "slice_width must be in 0..32");
      net->opt.slice_width = cfg->slice_width;
      if (cfg->order_weight < 0 || cfg->order_weight > 1000)
        return set_err(QTN_EINVAL, "order_weight must be in 0..1000");
      net->opt.order_weight = cfg->order_weight;
      if (cfg->hybrid_width < 0 || cfg->hybrid_width > kMaxWidth)
        return set_err(QTN_EINVAL, "hybrid_width must be in 0..32");
      if (cfg->hybrid_width > 0) net->hybrid_width = cfg->hybrid_width;
    }
    const int m = (int)n_edges;
    net->cones.resize(m);
    net->minfill.resize(m);
    qtn_network *raw = net.get();
    parallel_for(m, [&](int e) { raw->cones[e] = build_lightcone(raw->g, e, p); });
    *out = net.release();
    return QTN_OK;
  } catch (const std::bad_alloc &) {
    return set_err(QTN_ENOMEM, "host allocation failed");
  } catch (const std::exception &e) {
    return set_err(QTN_EINVAL, e.what());
  } catch (...) {
    return exception_status();
  }
}

int qtn_network_info(const qtn_network *cnet, int64_t edge, int32_t *n_vars, int32_t *n_tensors,
                     int32_t *width_minfill) {
  try {
    auto *net = const_cast<qtn_network *>(cnet);
    if (!net) return set_err(QTN_EINVAL, "network is NULL");
    if (edge < 0 || edge >= (int64_t)net->cones.size())
      return set_err(QTN_EINVAL, "edge out of range");
    const LightCone &lc = net->cones[edge];
    int32_t w = 0;
    if (width_minfill) {
      PlanOptions o = net->opt;
      o.max_levels = 1;
      o.max_width = 64;
      ConePlan pl;
      std::string err = plan_cone(lc, get_minfill(net, (int)edge), o, &pl);
      if (!err.empty()) return set_err(QTN_EINVAL, err);
      w = pl.max_width;
    }
    if (n_vars) *n_vars = lc.n_vars;
    if (n_tensors) *n_tensors = (int32_t)lc.gates.size();
    if (width_minfill) *width_minfill = w;
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_order_minfill(const qtn_network *cnet, int64_t edge, int32_t *order_out) {
  try {
    auto *net = const_cast<qtn_network *>(cnet);
    if (!net || !order_out) return set_err(QTN_EINVAL, "NULL argument");
    if (edge < 0 || edge >= (int64_t)net->cones.size())
      return set_err(QTN_EINVAL, "edge out of range");
    const auto &o = get_minfill(net, (int)edge);
    std::copy(o.begin(), o.end(), order_out);
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_plan(qtn_network *net, const int32_t *const *orders, int32_t precision,
             size_t *workspace_bytes_out) {
  try {
    if (!net) return set_err(QTN_EINVAL, "network is NULL");
    if (precision != QTN_C128 && precision != QTN_C64 && precision != QTN_MIXED)
      return set_err(QTN_EINVAL, "precision must be QTN_C128, QTN_C64 or QTN_MIXED");
    const int m = (int)net->cones.size();
    std::vector<ConePlan> plans(m);
    std::vector<std::string> errs(m);
    PlanOptions o = net->opt;
    o.precision = precision;
    parallel_for(m, [&](int e) {
      const LightCone &lc = net->cones[e];
      const bool given = orders && orders[e];
      std::vector<int> ord;
      // order search by the merged plan's cost (order_weight > 0) or by the
      // sum of 2^width
      const PlanOptions *cost_opt = o.order_weight > 0 ? &o : nullptr;
      if (given)
        ord.assign(orders[e], orders[e] + lc.n_vars);
      else if (net->order_trials > 1)
        ord = search_order(lc, net->order_trials, cost_opt, o.order_weight);
      else
        ord = get_minfill(net, e);
      if (o.slice_width > 0 && order_width(lc, ord) > o.slice_width) {
        // index slicing: fix variables until the widest bucket fits the cap,
        // then plan the restricted light cone (a caller's order still applies:
        // the fixed variables are left with empty buckets)
        std::vector<int> cord;
        const std::vector<int> sv = choose_slices(lc, o.slice_width, kMaxSliceVars,
                                                  net->order_trials, &cord, cost_opt, o.order_weight);
        LightCone sc = lc;
        for (size_t k = 0; k < sv.size(); k++) sc = slice_cone(sc, sv[k], (int)k);
        if (!given) {
          // the full order search, unless it is wider than the order the
          // choice of slices reached
          ord = net->order_trials > 1 ? search_order(sc, net->order_trials, cost_opt, o.order_weight)
                                      : minfill_order(sc);
          if (order_width(sc, ord) > std::max(o.slice_width, order_width(sc, cord))) ord = cord;
        }
        errs[e] = plan_cone(sc, ord, o, &plans[e]);
        plans[e].slice_vars = sv;
        plans[e].n_slices = 1 << sv.size();
        plans[e].gates = sc.gates;
        return;
      }
      errs[e] = plan_cone(lc, ord, o, &plans[e]);
    });
    for (int e = 0; e < m; e++)
      if (!errs[e].empty()) {
        bool range = errs[e].find("exceeds") != std::string::npos;
        return set_err(range ? QTN_ERANGE : QTN_EINVAL, "edge " + std::to_string(e) + ": " + errs[e]);
      }
    auto ex = std::make_unique<Exec>();
    net->plans.swap(plans);
    net->precision = precision;
    qtn_network *one[1] = {net};
    int rc = build_schedule(one, 1, &ex->sched, nullptr, 0, 1,
                            net->executor == 2 || net->executor == 4 || net->executor == 5);
    if (rc) {
      net->plans.clear();
      net->planned = false;
      return rc;
    }
    drop_batches_with(net);
    ex->persistent = net->executor == 2 || net->executor == 4 || net->executor == 5;
    ex->hybrid = net->executor == 5;
    ex->dataflow = net->executor == 4;
    ex->lead_per_cone = net->executor == 3;
    {
      size_t mx = ex->sched.total;
      for (const Force &f : tune_candidates()) {
        Schedule tmp;
        if (build_schedule(one, 1, &tmp, &f, kTuneSingleWidth) == QTN_OK)
          mx = std::max(mx, tmp.total);
      }
      net->tune_workspace = mx;
    }
    ex->spin_limit = net->spin_limit;
    if (net->exec) ex->rt.take(net->exec->rt);
    net->exec = std::move(ex);
    net->planned = true;
    net->version++;
    if (workspace_bytes_out) *workspace_bytes_out = net->tune_workspace;
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_set_angles(qtn_network *net, const double *gamma, const double *beta) {
  if (!net || !gamma || !beta) return set_err(QTN_EINVAL, "NULL argument");
  if (!finite_angles(net->p, gamma, beta)) return set_err(QTN_EINVAL, "angles must be finite");
  net->gamma.assign(gamma, gamma + net->p);
  net->beta.assign(beta, beta + net->p);
  return QTN_OK;
}

static int record_timing(qtn_network *net, const Exec &X, const Timer &tm, qtn_timing *timing);

static int contract_impl(qtn_network *net, void *ws, size_t bytes, void *stream, double *zz,
                         double *zz_im, double *energy, qtn_timing *timing) {
  try {
    if (!net) return set_err(QTN_EINVAL, "network is NULL");
    if (!net->planned) return set_err(QTN_ESTATE, "qtn_plan has not been called");
    Timer tm;
    tm.on = timing != nullptr;
    std::vector<double> res;
    int rc = run_exec(*net->exec, {net}, ws, bytes, stream, net->n_streams, net->eager, tm, res);
    if (rc) return rc;
    if (timing && (rc = record_timing(net, *net->exec, tm, timing))) return rc;
    const int m = net->exec->sched.n_cones;
    if (zz) std::copy(res.begin(), res.begin() + m, zz);
    if (zz_im) std::copy(res.begin() + m, res.begin() + 2 * m, zz_im);
    if (energy) *energy = res[2 * m];
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

// The launch log and per-class totals of a timed run of X (bytes and flops
// cover every angle set of the run).
static int record_timing(qtn_network *net, const Exec &X, const Timer &tm, qtn_timing *timing) {
    qtn_timing t;
    std::memset(&t, 0, sizeof t);
    {
      net->launch_log.clear();
      const Schedule &sc = X.sched;
      for (auto &r : tm.recs) {
        float ms = 0;
        QTN_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        t.ms[r.kind] += ms;
        t.launches[r.kind]++;
        qtn_launch_rec lr;
        std::memset(&lr, 0, sizeof lr);
        lr.kind = r.kind;
        lr.group = r.group;
        lr.n_groups = r.n_groups;
        lr.ms = ms;
        lr.bytes = r.bytes;
        lr.flops = r.flops;
        if (r.group >= 0 && r.group < (int)sc.groups.size()) {
          const DevGroup &g = sc.groups[r.group];
          lr.w = g.w;
          lr.L = g.L;
          lr.n_ops = g.n_ops;
          lr.variant = g.variant;
          lr.n_units = (int32_t)g.n_units;
          lr.prec = g.prec;
          lr.cvt = g.cvt;
          lr.knob = g.variant == kVarStream || g.variant == kVarCell || g.variant == kVarMfma ? g.rls : 0;
          lr.serial = g.variant == kVarStream || g.variant == kVarCell ? g.sl : 0;
        }
        net->launch_log.push_back(lr);
      }
      for (int k = 0; k < QTN_NKERNELS; k++) {
        t.bytes[k] = X.sched.bytes[k] * X.sched.n_sets;
        t.flops[k] = X.sched.flops[k] * X.sched.n_sets;
      }
      if (X.persistent) {
        for (int k = 0; k < QTN_K_PERSISTENT; k++) {
          t.bytes[QTN_K_PERSISTENT] += t.bytes[k];
          t.flops[QTN_K_PERSISTENT] += t.flops[k];
          t.bytes[k] = t.flops[k] = 0;
        }
      }
    }
    *timing = t;
    return QTN_OK;
}

int qtn_contract(qtn_network *net, void *d_workspace, size_t bytes, void *hip_stream,
                 double *zz_out, double *zz_imag_out, double *energy_out) {
  return contract_impl(net, d_workspace, bytes, hip_stream, zz_out, zz_imag_out, energy_out,
                       nullptr);
}

constexpr int kMaxAngleSets = 1024;

static Exec *angle_exec(qtn_network *net, int n_sets, int *rc) {
  if (net->angle_exec && net->angle_sets == n_sets && net->angle_version == net->version)
    return net->angle_exec.get();
  auto ex = std::make_unique<Exec>();
  qtn_network *one[1] = {net};
  // the same kernel mappings as the network's own schedule (so that every
  // set equals its single-set evaluation), though launched per group
  *rc = build_schedule(one, 1, &ex->sched, nullptr, 0, n_sets, net->exec->persistent);
  if (*rc) return nullptr;
  // per-group launches (the persistent executors run one set)
  ex->lead_per_cone = net->executor == 3;
  ex->spin_limit = net->spin_limit;
  if (net->angle_exec) ex->rt.take(net->angle_exec->rt);
  net->angle_exec = std::move(ex);
  net->angle_sets = n_sets;
  net->angle_version = net->version;
  return net->angle_exec.get();
}

int qtn_angles_workspace(qtn_network *net, int32_t n_sets, size_t *bytes_out) {
  try {
    if (!net || !bytes_out) return set_err(QTN_EINVAL, "NULL argument");
    if (!net->planned) return set_err(QTN_ESTATE, "qtn_plan has not been called");
    if (n_sets < 1 || n_sets > kMaxAngleSets)
      return set_err(QTN_EINVAL, "n_sets must be in 1.." + std::to_string(kMaxAngleSets));
    int rc = QTN_OK;
    Exec *ex = angle_exec(net, n_sets, &rc);
    if (!ex) return rc;
    *bytes_out = ex->sched.total;
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_contract_angles(qtn_network *net, void *d_workspace, size_t bytes, void *hip_stream,
                        int32_t n_sets, const double *gamma, const double *beta, double *zz_out,
                        double *energy_out, qtn_timing *timing) {
  try {
    if (!net || !gamma || !beta) return set_err(QTN_EINVAL, "NULL argument");
    if (!net->planned) return set_err(QTN_ESTATE, "qtn_plan has not been called");
    if (n_sets < 1 || n_sets > kMaxAngleSets)
      return set_err(QTN_EINVAL, "n_sets must be in 1.." + std::to_string(kMaxAngleSets));
    const int p = net->p;
    std::vector<double> ang((size_t)n_sets * 2 * p);
    for (int k = 0; k < n_sets; k++) {
      if (!finite_angles(p, gamma + (size_t)k * p, beta + (size_t)k * p))
        return set_err(QTN_EINVAL, "angles of set " + std::to_string(k) + " are not finite");
      std::copy(gamma + (size_t)k * p, gamma + (size_t)(k + 1) * p, ang.begin() + (size_t)k * 2 * p);
      std::copy(beta + (size_t)k * p, beta + (size_t)(k + 1) * p,
                ang.begin() + (size_t)k * 2 * p + p);
    }
    int rc = QTN_OK;
    Exec *ex = angle_exec(net, n_sets, &rc);
    if (!ex) return rc;
    Timer tm;
    tm.on = timing != nullptr;
    std::vector<double> res;
    rc = run_exec(*ex, {net}, d_workspace, bytes, hip_stream, net->n_streams, net->eager, tm, res,
                  ang.data());
    if (rc) return rc;
    if (timing && (rc = record_timing(net, *ex, tm, timing))) return rc;
    const int m = (int)net->cones.size(), per = 2 * m + 1;
    for (int k = 0; k < n_sets; k++) {
      if (zz_out) std::copy(res.begin() + (size_t)k * per, res.begin() + (size_t)k * per + m,
                            zz_out + (size_t)k * m);
      if (energy_out) energy_out[k] = res[(size_t)k * per + 2 * m];
    }
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_contract_timed(qtn_network *net, void *d_workspace, size_t bytes, void *hip_stream,
                       double *zz_out, double *energy_out, qtn_timing *timing) {
  if (!timing) return set_err(QTN_EINVAL, "timing is NULL");
  return contract_impl(net, d_workspace, bytes, hip_stream, zz_out, nullptr, energy_out, timing);
}

static Exec *batch_exec(qtn_network *const *nets, int32_t n, int *rc) {
  std::vector<std::pair<const qtn_network *, uint64_t>> key;
  for (int i = 0; i < n; i++) {
    if (!nets[i]) {
      *rc = set_err(QTN_EINVAL, "NULL network in batch");
      return nullptr;
    }
    if (!nets[i]->planned) {
      *rc = set_err(QTN_ESTATE, "network " + std::to_string(i) + " is not planned");
      return nullptr;
    }
    key.push_back({nets[i], nets[i]->version});
  }
  std::lock_guard<std::mutex> lk(g_batch_lock);
  auto it = g_batch.find(key);
  if (it != g_batch.end()) return it->second.get();
  auto ex = std::make_unique<Exec>();
  *rc = build_schedule(nets, n, &ex->sched, nullptr, 0, 1,
                       nets[0]->executor != 1 && nets[0]->executor != 3);
  if (*rc) return nullptr;
  // batches default to the persistent executor
  ex->persistent = nets[0]->executor != 1 && nets[0]->executor != 3;
  ex->dataflow = nets[0]->executor == 4;
  ex->hybrid = nets[0]->executor == 5;
  ex->spin_limit = nets[0]->spin_limit;
  Exec *raw = ex.get();
  g_batch[key] = std::move(ex);
  return raw;
}

int qtn_batch_workspace(qtn_network *const *nets, int32_t n, size_t *workspace_bytes_out) {
  try {
    if (!nets || n < 1 || !workspace_bytes_out) return set_err(QTN_EINVAL, "bad batch arguments");
    int rc = QTN_OK;
    Exec *ex = batch_exec(nets, n, &rc);
    if (!ex) return rc;
    *workspace_bytes_out = ex->sched.total;
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_contract_batch(qtn_network *const *nets, int32_t n, void *d_workspace, size_t bytes,
                       void *hip_stream, double *zz_out, double *energy_out) {
  try {
    if (!nets || n < 1) return set_err(QTN_EINVAL, "bad batch arguments");
    int rc = QTN_OK;
    Exec *ex = batch_exec(nets, n, &rc);
    if (!ex) return rc;
    std::vector<const qtn_network *> list(nets, nets + n);
    Timer tm;
    std::vector<double> res;
    rc = run_exec(*ex, list, d_workspace, bytes, hip_stream, nets[0]->n_streams, nets[0]->eager,
                  tm, res);
    if (rc) return rc;
    const int m = ex->sched.n_cones;
    if (zz_out) std::copy(res.begin(), res.begin() + m, zz_out);
    if (energy_out) std::copy(res.begin() + 2 * m, res.begin() + 2 * m + n, energy_out);
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_autotune_batch(qtn_network *const *nets, int32_t n, void *d_workspace, size_t bytes,
                       void *hip_stream, qtn_batch_tune_report *report) {
  try {
    if (!nets || n < 1) return set_err(QTN_EINVAL, "bad batch arguments");
    int rc = QTN_OK;
    Exec *ex = batch_exec(nets, n, &rc);
    if (!ex) return rc;
    if (!ex->persistent || ex->dataflow)
      return set_err(QTN_ESTATE, "batch autotuning needs the persistent lockstep or hybrid executor");
    std::vector<const qtn_network *> list(nets, nets + n);
    struct Cand {
      int quarters, order;
    };
    std::vector<Cand> cands;
    for (int order = 0; order < 2; order++)
      for (int q : {4, 3, 2}) cands.push_back({q, order});
    auto apply = [&](const Cand &c) {
      ex->grid_quarters = c.quarters;
      set_item_order(ex->sched, c.order);
      drop_graph(ex->rt);
    };
    std::vector<double> best(cands.size(), 1e300);
    std::vector<int> grid(cands.size(), 0);
    for (size_t i = 0; i < cands.size(); i++) {
      apply(cands[i]);
      // the first call captures the graph (or warms up): not timed
      for (int r = 0; r < 4; r++) {
        Timer tm;
        std::vector<double> res;
        const auto t0 = std::chrono::steady_clock::now();
        rc = run_exec(*ex, list, d_workspace, bytes, hip_stream, nets[0]->n_streams,
                      nets[0]->eager, tm, res);
        const auto t1 = std::chrono::steady_clock::now();
        if (rc) {
          apply(cands[0]);
          return rc;
        }
        if (r > 0) best[i] = std::min(best[i], std::chrono::duration<double, std::milli>(t1 - t0).count());
      }
      grid[i] = persist_grid(*ex);
    }
    // the built configuration unless another is more than 3% faster
    size_t pick = 0;
    for (size_t i = 1; i < cands.size(); i++)
      if (best[i] < best[pick]) pick = i;
    if (best[0] <= 1.03 * best[pick]) pick = 0;
    apply(cands[pick]);
    if (report) {
      qtn_batch_tune_report r;
      std::memset(&r, 0, sizeof r);
      r.n_candidates = (int32_t)cands.size();
      r.pick = (int32_t)pick;
      for (size_t i = 0; i < cands.size(); i++) {
        r.grid_blocks[i] = grid[i];
        r.item_order[i] = cands[i].order;
        r.ms[i] = best[i];
      }
      *report = r;
    }
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

// Workspace of autotuning over n_sets copies of the network's angles: the
// largest candidate schedule.
static int tune_workspace_bytes(qtn_network *net, int n_sets, size_t *bytes) {
  if (n_sets == 1) {
    *bytes = net->tune_workspace;
    return QTN_OK;
  }
  qtn_network *one[1] = {net};
  size_t mx = 0;
  for (const Force &f : tune_candidates()) {
    Schedule tmp;
    const int rc = build_schedule(one, 1, &tmp, &f, kTuneSingleWidth, n_sets);
    if (rc) return rc;
    mx = std::max(mx, tmp.total);
  }
  *bytes = mx;
  return QTN_OK;
}

// The autotuner; every candidate runs over n_sets copies of the network's
// current angles (n_sets 1: one evaluation).
static int autotune_sets(qtn_network *net, void *d_workspace, size_t bytes, void *hip_stream,
                         int n_sets, qtn_tune_report *report) {
  try {
    if (!net) return set_err(QTN_EINVAL, "network is NULL");
    if (!net->planned) return set_err(QTN_ESTATE, "qtn_plan has not been called");
    if (n_sets < 1 || n_sets > kMaxAngleSets)
      return set_err(QTN_EINVAL, "n_sets must be in 1.." + std::to_string(kMaxAngleSets));
    size_t need = 0;
    int wrc = tune_workspace_bytes(net, n_sets, &need);
    if (wrc) return wrc;
    if (bytes < need)
      return set_err(QTN_ENOMEM, "autotuning needs a workspace of " + std::to_string(need) +
                                     " bytes");
    // the angles of every set: the network's current ones
    std::vector<double> set_angles;
    if (n_sets > 1)
      for (int k = 0; k < n_sets; k++) {
        set_angles.insert(set_angles.end(), net->gamma.begin(), net->gamma.end());
        set_angles.insert(set_angles.end(), net->beta.begin(), net->beta.end());
      }
    const auto &cands = tune_candidates();
    const int nc = (int)cands.size();
    qtn_network *one[1] = {net};
    // per plan group: measured ms per candidate, own launch and inside a block
    // (the fastest of the passes)
    struct Meas {
      double wide[8], block[8];
    };
    std::map<std::pair<int, int>, Meas> meas;
    qtn_tune_report rep;
    std::memset(&rep, 0, sizeof rep);
    rep.n_candidates = nc;
    // one runtime for every candidate: the network's own streams
    Exec ex;
    ex.rt.take(net->exec->rt);
    auto give_back = [&]() { net->exec->rt.take(ex.rt); };
    constexpr int kPasses = 2;
    for (int pass = 0; pass < kPasses; pass++)
      for (int ci = 0; ci < nc; ci++) {
        int rc = build_schedule(one, 1, &ex.sched, &cands[ci], kTuneSingleWidth, n_sets);
        if (rc) {
          give_back();
          return rc;
        }
        ex.rt.forget_schedule();
        Timer tm;
        tm.on = true;
        std::vector<double> res;
        rc = run_exec(ex, {net}, d_workspace, bytes, hip_stream, 1, true, tm, res,
                      n_sets > 1 ? set_angles.data() : nullptr);
        if (rc) {
          give_back();
          return rc;
        }
        // the same groups again, each alone in one workgroup
        Timer tb;
        tb.on = true;
        char *ws = (char *)d_workspace;
        const Schedule &s = ex.sched;
        for (size_t i = 0; i < s.singles.size(); i++) {
          // the cell mapping, the complex128 matrix form and matrix-form
          // tiles wider than one column block only run in their own launch
          const DevGroup &dg = s.groups[s.singles[i]];
          if (dg.variant == kVarCell || (dg.variant == kVarMfma && (dg.prec == 0 || dg.rls != 1)))
            continue;
          if ((rc = tb.begin(QTN_K_BLOCK, ex.rt.main, s.singles[i], 1, 0, 0, true))) {
            give_back();
            return rc;
          }
          hipError_t he = launch_block_groups(
              s.prec, ws + s.off_data, (const DevGroup *)(ws + s.off_groups),
              (const DevOp *)(ws + s.off_ops), (const int32_t *)(ws + s.off_stab),
              (const uint8_t *)(ws + s.off_uperm), (const int2 *)(ws + s.off_ranges),
              s.singles_range0 + (int)i, 1, n_sets, ex.rt.main, tb.t0(), tb.t1());
          if (he == hipSuccess) rc = tb.end(ex.rt.main, true);
          if (he != hipSuccess || rc) {
            give_back();
            return he != hipSuccess ? set_err(QTN_EDEVICE, hipGetErrorString(he)) : rc;
          }
        }
        hipError_t he = hipStreamSynchronize(ex.rt.main);
        if (he != hipSuccess) {
          give_back();
          return set_err(QTN_EDEVICE, std::string("autotune: ") + hipGetErrorString(he));
        }
        auto key_of = [&](int g) { return std::make_pair(s.group_cone[g], s.group_index[g]); };
        // a candidate only counts for the groups that ran its kernel
        auto ran = [&](int g) {
          if (cands[ci].variant == 3) return s.groups[g].variant == kVarMfma;
          if (cands[ci].variant == 4) return s.groups[g].variant == kVarCell;
          return true;
        };
        auto slot = [&](int g) -> Meas & {
          return meas.emplace(key_of(g), Meas{{-1, -1, -1, -1, -1, -1, -1, -1},
                                              {-1, -1, -1, -1, -1, -1, -1, -1}})
              .first->second;
        };
        auto keep_min = [](double &dst, double v) { dst = dst < 0 ? v : std::min(dst, v); };
        for (auto &r : tm.recs) {
          if (r.kind != QTN_K_WIDE || !ran(r.group)) continue;
          float ms = 0;
          (void)hipEventElapsedTime(&ms, r.a, r.b);
          keep_min(slot(r.group).wide[ci], ms);
        }
        for (auto &r : tb.recs) {
          if (!ran(r.group)) continue;
          float ms = 0;
          (void)hipEventElapsedTime(&ms, r.a, r.b);
          keep_min(slot(r.group).block[ci], ms);
        }
      }
    for (auto &kv : meas)
      for (int ci = 0; ci < nc; ci++)
        if (kv.second.wide[ci] > 0) rep.cand_ms[ci] += kv.second.wide[ci];
    // per group: the fastest candidate for where the width rule places it;
    // the width rule's own configuration is kept unless another is faster by
    // more than the tolerance (near-ties are timing noise and would make the
    // tuned schedule differ from run to run).  Every group's timings go to
    // the tuning log.
    constexpr double kSwitchGain = 0.97;
    net->tune_log.clear();
    for (auto &kv : meas) {
      ConePlan &pl = net->plans[kv.first.first];
      Group &G = pl.groups[kv.first.second];
      const Meas &m = kv.second;
      const double *t = G.small ? m.block : m.wide;
      const int rls = std::min(G.L - 1, net->lane_sum_bits), sl = G.L - 1 - rls;
      const bool rule_stream = (int)G.ops.size() <= kStreamMaxOps && sl <= kStreamMaxSerial &&
                               sl >= 2 && net->variant != 1 &&
                               max_operand_bytes(G, pl) <= kOffset32Bytes;
      // the rule's own configuration: the cell mapping wherever it ran (own
      // launches of the per-group executors), else streaming or generic
      int rule_cell = -1;
      for (int ci = 0; ci < nc; ci++)
        if (!G.small && !net->exec->persistent && net->variant != 1 && net->variant != 2 &&
            cands[ci].variant == 4 && cands[ci].rls == kCellRuleCB && t[ci] >= 0)
          rule_cell = ci;
      int best = rule_cell;
      for (int ci = 0; ci < nc && rule_cell < 0; ci++)
        if (cands[ci].variant == (rule_stream ? 2 : 1) && (rule_stream ? cands[ci].rls == rls : true))
          if (t[ci] >= 0) best = ci;
      for (int ci = 0; ci < nc; ci++)
        if (t[ci] >= 0 && (best < 0 || t[ci] < kSwitchGain * t[best])) best = ci;
      if (best >= 0) {
        G.pick_variant = (int8_t)cands[best].variant;
        G.pick_rls = (int8_t)cands[best].rls;
        if (!G.small) {
          rep.tuned_ms += t[best];
          rep.picks[best]++;
          rep.n_groups++;
        }
      }
      qtn_tune_rec tr;
      std::memset(&tr, 0, sizeof tr);
      group_features(G, pl, net->precision, tr.features);
      double mb = -1, ms_stream = -1, ms_mfma = -1;
      for (int ci = 0; ci < nc; ci++) {
        if (m.block[ci] >= 0 && (mb < 0 || m.block[ci] < mb)) mb = m.block[ci];
        if ((cands[ci].variant == 2 || cands[ci].variant == 4) && m.wide[ci] >= 0 &&
            (ms_stream < 0 || m.wide[ci] < ms_stream))
          ms_stream = m.wide[ci];
        if (cands[ci].variant == 3) ms_mfma = m.wide[ci];
      }
      tr.ms[QTN_VAR_BLOCK] = mb;
      tr.ms[QTN_VAR_STREAM] = ms_stream;
      tr.ms[QTN_VAR_GENERIC] = m.wide[0];
      tr.ms[QTN_VAR_MFMA] = ms_mfma;
      net->tune_log.push_back(tr);
    }
    // the tuned schedule replaces the current one, on the same streams
    auto tuned = std::make_unique<Exec>();
    int rc = build_schedule(one, 1, &tuned->sched, nullptr, 0, 1, net->exec->persistent);
    if (rc) {
      give_back();
      return rc;
    }
    tuned->persistent = net->exec->persistent;
    tuned->hybrid = net->exec->hybrid;
    tuned->dataflow = net->exec->dataflow;
    tuned->lead_per_cone = net->exec->lead_per_cone;
    tuned->spin_limit = net->exec->spin_limit;
    tuned->rt.take(ex.rt);
    drop_batches_with(net);
    net->exec = std::move(tuned);
    net->version++;
    if (report) *report = rep;
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

// FNV-1a over a group's width, summed count and operand index sets.
static uint32_t group_shape(const Group &G) {
  uint32_t h = 2166136261u;
  auto mix = [&](uint32_t v) {
    for (int k = 0; k < 4; k++) {
      h ^= (v >> (8 * k)) & 0xFFu;
      h *= 16777619u;
    }
  };
  mix((uint32_t)G.w);
  mix((uint32_t)G.L);
  mix((uint32_t)G.ops.size());
  for (const Operand &o : G.ops) {
    mix(o.mask);
    mix((uint32_t)o.level);
  }
  return h;
}

int qtn_tune_picks(const qtn_network *net, int64_t cap, qtn_tune_pick *out, int64_t *n_out) {
  if (!net || !n_out || (cap > 0 && !out)) return set_err(QTN_EINVAL, "NULL argument");
  if (!net->planned) return set_err(QTN_ESTATE, "qtn_plan has not been called");
  int64_t n = 0;
  for (size_t e = 0; e < net->plans.size(); e++)
    for (size_t g = 0; g < net->plans[e].groups.size(); g++, n++) {
      if (n >= cap) continue;
      const Group &G = net->plans[e].groups[g];
      qtn_tune_pick p;
      std::memset(&p, 0, sizeof p);
      p.edge = (int32_t)e;
      p.group = (int32_t)g;
      p.place = G.pick_place;
      p.variant = G.pick_variant;
      p.rls = G.pick_rls;
      p.shape = group_shape(G);
      out[n] = p;
    }
  *n_out = n;
  return QTN_OK;
}

int qtn_set_tune_picks(qtn_network *net, const qtn_tune_pick *picks, int64_t n) {
  try {
    if (!net || (n > 0 && !picks)) return set_err(QTN_EINVAL, "NULL argument");
    if (!net->planned) return set_err(QTN_ESTATE, "qtn_plan has not been called");
    for (int64_t i = 0; i < n; i++) {
      const qtn_tune_pick &p = picks[i];
      if (p.edge < 0 || p.edge >= (int32_t)net->plans.size() || p.group < 0 ||
          p.group >= (int32_t)net->plans[p.edge].groups.size())
        return set_err(QTN_EINVAL, "pick " + std::to_string(i) + " names no group of this plan");
      if (group_shape(net->plans[p.edge].groups[p.group]) != p.shape)
        return set_err(QTN_EINVAL, "pick " + std::to_string(i) + " is for a different group");
      if (p.place < -1 || p.place > 1 || p.variant < -1 || p.variant > 4 || p.rls < -1 || p.rls > 5)
        return set_err(QTN_EINVAL, "pick " + std::to_string(i) + " is out of range");
    }
    for (int64_t i = 0; i < n; i++) {
      Group &G = net->plans[picks[i].edge].groups[picks[i].group];
      G.pick_place = picks[i].place;
      G.pick_variant = picks[i].variant;
      G.pick_rls = picks[i].rls;
    }
    qtn_network *one[1] = {net};
    auto ex = std::make_unique<Exec>();
    int rc = build_schedule(one, 1, &ex->sched, nullptr, 0, 1, net->exec->persistent);
    if (rc) return rc;
    ex->rt.take(net->exec->rt);
    ex->persistent = net->exec->persistent;
    ex->hybrid = net->exec->hybrid;
    ex->dataflow = net->exec->dataflow;
    ex->lead_per_cone = net->exec->lead_per_cone;
    ex->spin_limit = net->exec->spin_limit;
    drop_batches_with(net);
    net->exec = std::move(ex);
    net->version++;
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_autotune(qtn_network *net, void *d_workspace, size_t bytes, void *hip_stream,
                 qtn_tune_report *report) {
  return autotune_sets(net, d_workspace, bytes, hip_stream, 1, report);
}

int qtn_gradient_workspace(qtn_network *net, size_t *workspace_bytes_out) {
  if (!net) return set_err(QTN_EINVAL, "NULL argument");
  return qtn_angles_workspace(net, 4 * net->p + 1, workspace_bytes_out);
}

int qtn_energy_gradient(qtn_network *net, void *d_workspace, size_t bytes, void *hip_stream,
                        const double *gamma, const double *beta, double step, double *energy_out,
                        double *grad_gamma_out, double *grad_beta_out) {
  try {
    if (!net || !gamma || !beta || !energy_out || !grad_gamma_out || !grad_beta_out)
      return set_err(QTN_EINVAL, "NULL argument");
    if (!(step > 0.0) || !std::isfinite(step))
      return set_err(QTN_EINVAL, "step must be positive and finite");
    const int p = net->p, n = 4 * p + 1;
    // set 0: the angles; then gamma_l + h, gamma_l - h for every l, then the
    // same for beta_l
    std::vector<double> g((size_t)n * p), b((size_t)n * p), e(n);
    for (int k = 0; k < n; k++) {
      std::copy(gamma, gamma + p, g.begin() + (size_t)k * p);
      std::copy(beta, beta + p, b.begin() + (size_t)k * p);
    }
    for (int l = 0; l < p; l++) {
      g[(size_t)(1 + 2 * l) * p + l] += step;
      g[(size_t)(2 + 2 * l) * p + l] -= step;
      b[(size_t)(1 + 2 * p + 2 * l) * p + l] += step;
      b[(size_t)(2 + 2 * p + 2 * l) * p + l] -= step;
    }
    const int rc = qtn_contract_angles(net, d_workspace, bytes, hip_stream, n, g.data(), b.data(),
                                       nullptr, e.data(), nullptr);
    if (rc) return rc;
    *energy_out = e[0];
    for (int l = 0; l < p; l++) {
      grad_gamma_out[l] = (e[1 + 2 * l] - e[2 + 2 * l]) / (2.0 * step);
      grad_beta_out[l] = (e[1 + 2 * p + 2 * l] - e[2 + 2 * p + 2 * l]) / (2.0 * step);
    }
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_tune_angles_workspace(qtn_network *net, int32_t n_sets, size_t *bytes_out) {
  try {
    if (!net || !bytes_out) return set_err(QTN_EINVAL, "NULL argument");
    if (!net->planned) return set_err(QTN_ESTATE, "qtn_plan has not been called");
    if (n_sets < 1 || n_sets > kMaxAngleSets)
      return set_err(QTN_EINVAL, "n_sets must be in 1.." + std::to_string(kMaxAngleSets));
    return tune_workspace_bytes(net, n_sets, bytes_out);
  } catch (...) {
    return exception_status();
  }
}

int qtn_autotune_angles(qtn_network *net, void *d_workspace, size_t bytes, void *hip_stream,
                        int32_t n_sets, qtn_tune_report *report) {
  return autotune_sets(net, d_workspace, bytes, hip_stream, n_sets, report);
}

int qtn_tune_log(const qtn_network *net, int64_t cap, qtn_tune_rec *out, int64_t *n_out) {
  if (!net || !n_out || (cap > 0 && !out)) return set_err(QTN_EINVAL, "NULL argument");
  const auto &lg = net->tune_log;
  const int64_t n = std::min<int64_t>(cap, (int64_t)lg.size());
  for (int64_t i = 0; i < n; i++) out[i] = lg[i];
  *n_out = (int64_t)lg.size();
  return QTN_OK;
}

int qtn_launch_log(const qtn_network *net, int64_t cap, qtn_launch_rec *out, int64_t *n_out) {
  if (!net || !n_out || (cap > 0 && !out)) return set_err(QTN_EINVAL, "NULL argument");
  const auto &lg = net->launch_log;
  const int64_t n = std::min<int64_t>(cap, (int64_t)lg.size());
  for (int64_t i = 0; i < n; i++) out[i] = lg[i];
  *n_out = (int64_t)lg.size();
  return QTN_OK;
}

int qtn_get_plan_stats(const qtn_network *net, qtn_plan_stats *out) {
  if (!net || !out) return set_err(QTN_EINVAL, "NULL argument");
  if (!net->planned) return set_err(QTN_ESTATE, "qtn_plan has not been called");
  qtn_plan_stats st;
  std::memset(&st, 0, sizeof st);
  for (const ConePlan &pl : net->plans) {
    st.n_buckets += pl.n_buckets;
    st.n_groups += (int64_t)pl.groups.size();
    for (const Group &G : pl.groups) st.n_wide += G.small ? 0 : 1;
    st.max_width = std::max(st.max_width, pl.max_width);
    for (int w : pl.bucket_width)
      if (w > 0 && w < 40) st.width_hist[w]++;
    st.paper_flops += pl.paper_flops * pl.n_slices;
    st.n_sliced += pl.n_slices > 1 ? 1 : 0;
    st.n_slices += pl.n_slices;
  }
  const Schedule &s = net->exec->sched;
  for (int k = 0; k < QTN_NKERNELS; k++) {
    st.bytes += s.bytes[k];
    st.flops += s.flops[k];
  }
  st.workspace = s.total;
  for (size_t gi = 0; gi < s.groups.size(); gi++) {
    const DevGroup &g = s.groups[gi];
    st.n_matrix += g.variant == kVarMfma ? 1 : 0;
    st.n_cell += g.variant == kVarCell ? 1 : 0;
    st.n_stream += g.variant == kVarStream ? 1 : 0;
    const ConePlan &pl = net->plans[s.group_cone[gi]];
    if (max_operand_bytes(pl.groups[s.group_index[gi]], pl) > kOffset32Bytes) {
      st.n_over4g++;
      st.n_over4g_generic += g.variant == kVarGeneric ? 1 : 0;
    }
  }
  *out = st;
  return QTN_OK;
}

int qtn_slice_vars(const qtn_network *net, int64_t edge, int32_t cap, int32_t *vars_out,
                   int32_t *n_out) {
  if (!net || !n_out || (cap > 0 && !vars_out)) return set_err(QTN_EINVAL, "NULL argument");
  if (!net->planned) return set_err(QTN_ESTATE, "qtn_plan has not been called");
  if (edge < 0 || edge >= (int64_t)net->plans.size()) return set_err(QTN_EINVAL, "edge out of range");
  const auto &sv = net->plans[edge].slice_vars;
  for (int k = 0; k < (int)sv.size() && k < cap; k++) vars_out[k] = sv[k];
  *n_out = (int32_t)sv.size();
  return QTN_OK;
}

int qtn_plan_order(const qtn_network *net, int64_t edge, int32_t *order_out) {
  if (!net || !order_out) return set_err(QTN_EINVAL, "NULL argument");
  if (!net->planned) return set_err(QTN_ESTATE, "qtn_plan has not been called");
  if (edge < 0 || edge >= (int64_t)net->plans.size()) return set_err(QTN_EINVAL, "edge out of range");
  const auto &o = net->plans[edge].order;
  std::copy(o.begin(), o.end(), order_out);
  return QTN_OK;
}

}  // extern "C"

// One bucket contraction of caller-given tensors: a one-group schedule whose
// descriptors address the caller's data buffer.
struct qtn_bucket {
  Schedule s;              // one group; s.desc_blob holds its descriptors
  DevGroup hg;             // host copy of the group record
  size_t off_groups = 0, off_ops = 0, off_stab = 0, off_uperm = 0;
  int64_t data_bytes = 0;  // end of the last tensor in the data buffer
  double bytes = 0, flops = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};  // timed runs: start/stop of the dispatch
  ~qtn_bucket() {
    for (hipEvent_t &e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace {

// Uploads the bucket's descriptors to `desc` (device) and runs its kernel
// on the caller's data buffer.
// t0, t1: events attached to the kernel's dispatch (timed runs), or null.
int bucket_run(const qtn_bucket *b, void *d_data, size_t data_bytes, char *desc, hipStream_t st,
               hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr) {
  if ((int64_t)data_bytes < b->data_bytes)
    return set_err(QTN_ENOMEM, "data buffer smaller than the bucket's tensors");
  if (((uintptr_t)d_data & 255u) != 0) return set_err(QTN_EINVAL, "data buffer not 256-byte aligned");
  QTN_HIP(hipMemcpyAsync(desc, b->s.desc_blob.data(), b->s.desc_blob.size(), hipMemcpyHostToDevice, st));
  QTN_HIP(launch_wide_group(b->hg, d_data, (const DevGroup *)(desc + b->off_groups),
                            (const DevOp *)(desc + b->off_ops), (const int32_t *)(desc + b->off_stab),
                            (const uint8_t *)(desc + b->off_uperm), 0, 1, st, t0, t1));
  return QTN_OK;
}

}  // namespace

extern "C" {

int qtn_bucket_plan(int32_t n_ops, const int32_t *ranks, const int32_t *labels,
                    const int64_t *offsets, int32_t n_out, const int32_t *out_labels,
                    int64_t out_offset, int32_t precision, int32_t variant, int32_t knob,
                    qtn_bucket **out) {
  if (!ranks || !labels || !offsets || !out || (n_out > 0 && !out_labels))
    return set_err(QTN_EINVAL, "NULL argument");
  if (n_ops < 1 || n_ops > 64) return set_err(QTN_EINVAL, "n_ops must be in 1..64");
  if (n_out < 0 || n_out > kMaxWidth) return set_err(QTN_EINVAL, "n_out must be in 0..32");
  if (precision != QTN_C128 && precision != QTN_C64)
    return set_err(QTN_EINVAL, "precision must be QTN_C128 or QTN_C64");
  if (variant < 0 || variant > 4) return set_err(QTN_EINVAL, "variant must be 0..4");
  try {
    // union order: the summed labels ascending, then the output labels
    std::map<int32_t, int> seen;  // label -> union position (-1 until placed)
    int64_t n_lab = 0;
    for (int k = 0; k < n_ops; k++) {
      if (ranks[k] < 0 || ranks[k] > kMaxWidth) return set_err(QTN_EINVAL, "operand rank out of range");
      for (int j = 0; j < ranks[k]; j++) seen[labels[n_lab + j]] = -1;
      n_lab += ranks[k];
    }
    for (int j = 0; j < n_out; j++) {
      auto it = seen.find(out_labels[j]);
      if (it == seen.end()) return set_err(QTN_EINVAL, "output label held by no operand");
      if (it->second != -1) return set_err(QTN_EINVAL, "repeated output label");
      it->second = -2;  // kept
    }
    int L = 0;
    for (auto &kv : seen)
      if (kv.second == -1) kv.second = L++;
    const int w = L + n_out;
    if (L < 1) return set_err(QTN_EINVAL, "no summed label: a bucket sums at least one index");
    if (L > kMaxLevels) return set_err(QTN_ERANGE, "more than 8 summed labels");
    if (w > kMaxWidth) return set_err(QTN_ERANGE, "union of more than 32 labels");
    for (int j = 0; j < n_out; j++) seen[out_labels[j]] = L + j;
    auto qb = std::make_unique<qtn_bucket>();
    const int64_t es = precision == QTN_C64 ? 8 : 16;
    ConePlan pl;
    Group G;
    G.w = w;
    G.L = L;
    G.prec = (int8_t)precision;
    std::vector<std::pair<int64_t, int64_t>> ranges;  // byte ranges of the inputs
    n_lab = 0;
    for (int k = 0; k < n_ops; k++) {
      uint32_t mask = 0;
      int prev = -1;
      for (int j = 0; j < ranks[k]; j++) {
        const int pos = seen[labels[n_lab + j]];
        if (pos <= prev)
          return set_err(QTN_EINVAL, "operand " + std::to_string(k) +
                                         ": labels repeated or not in union order (summed labels "
                                         "ascending, then the output labels in order)");
        prev = pos;
        mask |= 1u << pos;
      }
      n_lab += ranks[k];
      const int64_t size = es << ranks[k];
      if (offsets[k] < 0 || offsets[k] % es) return set_err(QTN_EINVAL, "operand offset not aligned");
      ranges.push_back({offsets[k], offsets[k] + size});
      qb->data_bytes = std::max(qb->data_bytes, offsets[k] + size);
      Tensor t;
      t.vars.assign(ranks[k], 0);
      t.offset = offsets[k];
      t.prec = (int8_t)precision;
      pl.tensors.push_back(t);
      // level: after the summed labels below the operand's lowest one
      const uint32_t summed = mask & ((1u << L) - 1u);
      const int level = summed ? __builtin_ctz(summed) : L - 1;
      G.ops.push_back({k, mask, level});
    }
    std::stable_sort(G.ops.begin(), G.ops.end(),
                     [](const Operand &a, const Operand &b) { return a.level < b.level; });
    const int64_t osize = es << n_out;
    if (out_offset < 0 || out_offset % es) return set_err(QTN_EINVAL, "output offset not aligned");
    for (auto &r : ranges)
      if (r.first < out_offset + osize && out_offset < r.second)
        return set_err(QTN_EINVAL, "output overlaps an operand");
    qb->data_bytes = std::max(qb->data_bytes, out_offset + osize);
    Tensor to;
    to.vars.assign(n_out, 0);
    to.offset = out_offset;
    to.prec = (int8_t)precision;
    pl.tensors.push_back(to);
    G.out_tensor = n_ops;
    GroupEnv env;
    env.out_off = out_offset;
    env.var_req = variant;
    env.rls_req = knob > 0 ? knob : (variant == 4 ? kCellRuleCB : 2);
    Schedule &s = qb->s;
    int rc = describe_group(G, pl, env, s, &qb->hg, &qb->bytes, &qb->flops);
    if (rc) return rc;
    if (qb->hg.n_units == 0 || qb->hg.n_units > 0x7FFFFFFFu)
      return set_err(QTN_ERANGE, "too many units for one launch");
    qb->hg.op_begin = 0;
    s.groups.assign(1, qb->hg);
    qb->off_groups = 0;
    qb->off_ops = align_up(sizeof(DevGroup), 256);
    qb->off_stab = align_up(qb->off_ops + sizeof(DevOp) * s.ops.size(), 256);
    qb->off_uperm = align_up(qb->off_stab + sizeof(int32_t) * s.stab.size(), 256);
    s.desc_blob.assign(align_up(qb->off_uperm + s.uperm.size(), 256), 0);
    std::memcpy(s.desc_blob.data() + qb->off_groups, s.groups.data(), sizeof(DevGroup));
    std::memcpy(s.desc_blob.data() + qb->off_ops, s.ops.data(), sizeof(DevOp) * s.ops.size());
    if (!s.stab.empty())
      std::memcpy(s.desc_blob.data() + qb->off_stab, s.stab.data(), sizeof(int32_t) * s.stab.size());
    std::memcpy(s.desc_blob.data() + qb->off_uperm, s.uperm.data(), s.uperm.size());
    *out = qb.release();
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_bucket_get_info(const qtn_bucket *b, qtn_bucket_info *out) {
  if (!b || !out) return set_err(QTN_EINVAL, "NULL argument");
  qtn_bucket_info r;
  std::memset(&r, 0, sizeof r);
  r.w = b->hg.w;
  r.L = b->hg.L;
  r.n_ops = b->hg.n_ops;
  r.variant = b->hg.variant;
  r.knob = b->hg.variant == kVarStream || b->hg.variant == kVarCell || b->hg.variant == kVarMfma ? b->hg.rls : 0;
  r.serial = b->hg.variant == kVarStream || b->hg.variant == kVarCell ? b->hg.sl : 0;
  r.n_units = b->hg.n_units;
  r.bytes = b->bytes;
  r.flops = b->flops;
  r.workspace_bytes = b->s.desc_blob.size();
  r.data_bytes = b->data_bytes;
  *out = r;
  return QTN_OK;
}

int qtn_bucket_contract(const qtn_bucket *b, void *d_data, size_t data_bytes, void *d_workspace,
                        size_t ws_bytes, void *hip_stream) {
  if (!b || !d_data || !d_workspace) return set_err(QTN_EINVAL, "NULL argument");
  if (ws_bytes < b->s.desc_blob.size()) return set_err(QTN_ENOMEM, "workspace too small");
  if (((uintptr_t)d_workspace & 255u) != 0) return set_err(QTN_EINVAL, "workspace not 256-byte aligned");
  try {
    return bucket_run(b, d_data, data_bytes, (char *)d_workspace, (hipStream_t)hip_stream);
  } catch (...) {
    return exception_status();
  }
}

int qtn_bucket_contract_timed(qtn_bucket *b, void *d_data, size_t data_bytes, void *d_workspace,
                              size_t ws_bytes, void *hip_stream, double *kernel_ms) {
  if (!b || !d_data || !d_workspace || !kernel_ms) return set_err(QTN_EINVAL, "NULL argument");
  if (ws_bytes < b->s.desc_blob.size()) return set_err(QTN_ENOMEM, "workspace too small");
  if (((uintptr_t)d_workspace & 255u) != 0) return set_err(QTN_EINVAL, "workspace not 256-byte aligned");
  try {
    for (hipEvent_t &e : b->ev)
      if (!e) QTN_HIP(hipEventCreate(&e));
    const int rc = bucket_run(b, d_data, data_bytes, (char *)d_workspace, (hipStream_t)hip_stream,
                              b->ev[0], b->ev[1]);
    if (rc) return rc;
    QTN_HIP(hipEventSynchronize(b->ev[1]));
    float ms = 0;
    QTN_HIP(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
    *kernel_ms = ms;
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_bucket_contract_noalloc(const qtn_bucket *b, void *d_data, size_t data_bytes,
                                void *hip_stream) {
  if (!b || !d_data) return set_err(QTN_EINVAL, "NULL argument");
  if (b->s.desc_blob.size() > kScratchBytes)
    return set_err(QTN_ERANGE, "bucket descriptors (" + std::to_string(b->s.desc_blob.size()) +
                                   " bytes) exceed the " + std::to_string(kScratchBytes) +
                                   "-byte device scratch");
  try {
    void *scr = nullptr;
    QTN_HIP(scratch_address(&scr));
    return bucket_run(b, d_data, data_bytes, (char *)scr, (hipStream_t)hip_stream);
  } catch (...) {
    return exception_status();
  }
}

void qtn_bucket_free(qtn_bucket *b) { delete b; }

int qtn_bucket_widths(const qtn_network *net, int64_t edge, int32_t *widths_out) {
  if (!net || !widths_out) return set_err(QTN_EINVAL, "NULL argument");
  if (!net->planned) return set_err(QTN_ESTATE, "qtn_plan has not been called");
  if (edge < 0 || edge >= (int64_t)net->plans.size()) return set_err(QTN_EINVAL, "edge out of range");
  const auto &w = net->plans[edge].bucket_width;
  std::copy(w.begin(), w.end(), widths_out);
  return QTN_OK;
}

}  // extern "C"

struct qtn_costmodel {
  std::vector<float> params, m1, m2;
  float mean[kMlpIn], inv_std[kMlpIn];
  bool norm_set = false;
  int step = 0;
};

namespace {

int mlp_upload_inputs(const qtn_costmodel *cm, const float *x, int64_t n, const MlpBuffers &b,
                      bool normalize, hipStream_t s, std::vector<float> &stage) {
  stage.assign(x, x + n * kMlpIn);
  if (normalize)
    for (int64_t i = 0; i < n; i++)
      for (int k = 0; k < kMlpIn; k++)
        stage[i * kMlpIn + k] = (stage[i * kMlpIn + k] - cm->mean[k]) * cm->inv_std[k];
  QTN_HIP(hipMemcpyAsync(b.x, stage.data(), sizeof(float) * n * kMlpIn, hipMemcpyHostToDevice, s));
  QTN_HIP(hipMemcpyAsync(b.params, cm->params.data(), sizeof(float) * kMlpParams,
                         hipMemcpyHostToDevice, s));
  return QTN_OK;
}

int mlp_check_ws(int64_t n, void *ws, size_t bytes) {
  if (n < 1) return set_err(QTN_EINVAL, "need at least one sample");
  if (!ws) return set_err(QTN_EINVAL, "workspace is NULL");
  if (bytes < mlp_buffers(ws, n).bytes) return set_err(QTN_ENOMEM, "cost-model workspace too small");
  return QTN_OK;
}

}  // namespace

extern "C" {

int qtn_costmodel_create(const float *params, qtn_costmodel **out) {
  if (!params || !out) return set_err(QTN_EINVAL, "NULL argument");
  try {
    auto *cm = new qtn_costmodel();
    cm->params.assign(params, params + kMlpParams);
    cm->m1.assign(kMlpParams, 0.0f);
    cm->m2.assign(kMlpParams, 0.0f);
    for (int k = 0; k < kMlpIn; k++) {
      cm->mean[k] = 0.0f;
      cm->inv_std[k] = 1.0f;
    }
    *out = cm;
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_costmodel_params(const qtn_costmodel *cm, float *params_out) {
  if (!cm || !params_out) return set_err(QTN_EINVAL, "NULL argument");
  std::copy(cm->params.begin(), cm->params.end(), params_out);
  return QTN_OK;
}

int qtn_costmodel_normalization(const qtn_costmodel *cm, float *mean_out, float *inv_std_out) {
  if (!cm || !mean_out || !inv_std_out) return set_err(QTN_EINVAL, "NULL argument");
  std::copy(cm->mean, cm->mean + kMlpIn, mean_out);
  std::copy(cm->inv_std, cm->inv_std + kMlpIn, inv_std_out);
  return QTN_OK;
}

int qtn_costmodel_workspace(int64_t n, size_t *bytes_out) {
  if (n < 1 || !bytes_out) return set_err(QTN_EINVAL, "bad arguments");
  *bytes_out = mlp_buffers(nullptr, n).bytes;
  return QTN_OK;
}

int qtn_costmodel_train(qtn_costmodel *cm, const float *x, const double *ms, int64_t n,
                        int32_t epochs, float lr, void *d_ws, size_t bytes, void *hip_stream,
                        float *loss_history) {
  try {
    if (!cm || !x || !ms || epochs < 1 || !(lr > 0)) return set_err(QTN_EINVAL, "bad arguments");
    int rc = mlp_check_ws(n, d_ws, bytes);
    if (rc) return rc;
    if (!cm->norm_set) {
      for (int k = 0; k < kMlpIn; k++) {
        double s = 0, s2 = 0;
        for (int64_t i = 0; i < n; i++) {
          s += x[i * kMlpIn + k];
          s2 += (double)x[i * kMlpIn + k] * x[i * kMlpIn + k];
        }
        const double mu = s / n, var = std::max(0.0, s2 / n - mu * mu);
        cm->mean[k] = (float)mu;
        cm->inv_std[k] = (float)(1.0 / std::max(1e-3, std::sqrt(var)));
      }
      cm->norm_set = true;
    }
    std::vector<float> t(n * kMlpOut), m(n * kMlpOut), stage;
    for (int64_t q = 0; q < n * kMlpOut; q++) {
      m[q] = ms[q] > 0 ? 1.0f : 0.0f;
      t[q] = ms[q] > 0 ? (float)std::log(ms[q]) : 0.0f;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    const MlpBuffers b = mlp_buffers(d_ws, n);
    if ((rc = mlp_upload_inputs(cm, x, n, b, true, s, stage))) return rc;
    QTN_HIP(hipMemcpyAsync(b.t, t.data(), sizeof(float) * n * kMlpOut, hipMemcpyHostToDevice, s));
    QTN_HIP(hipMemcpyAsync(b.m, m.data(), sizeof(float) * n * kMlpOut, hipMemcpyHostToDevice, s));
    QTN_HIP(hipMemcpyAsync(b.m1, cm->m1.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice, s));
    QTN_HIP(hipMemcpyAsync(b.m2, cm->m2.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice, s));
    float *hist = nullptr;
    QTN_HIP(hipHostMalloc((void **)&hist, sizeof(float) * epochs, hipHostMallocDefault));
    int step = cm->step;
    for (int e = 0; e < epochs; e++) {
      hipError_t he = mlp_loss_grad(b, (int)n, s);
      if (he == hipSuccess) he = hipMemcpyAsync(hist + e, b.loss, sizeof(float), hipMemcpyDeviceToHost, s);
      if (he == hipSuccess) he = mlp_adam(b, ++step, lr, s);
      if (he != hipSuccess) {
        (void)hipHostFree(hist);
        return set_err(QTN_EDEVICE, std::string("cost-model training: ") + hipGetErrorString(he));
      }
    }
    std::vector<float> p(kMlpParams), a(kMlpParams), q2(kMlpParams);
    hipError_t he = hipMemcpyAsync(p.data(), b.params, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipMemcpyAsync(a.data(), b.m1, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipMemcpyAsync(q2.data(), b.m2, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) {
      (void)hipHostFree(hist);
      return set_err(QTN_EDEVICE, std::string("cost-model training: ") + hipGetErrorString(he));
    }
    if (loss_history) std::copy(hist, hist + epochs, loss_history);
    (void)hipHostFree(hist);
    cm->params.swap(p);
    cm->m1.swap(a);
    cm->m2.swap(q2);
    cm->step = step;
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_costmodel_predict(const qtn_costmodel *cm, const float *x, int64_t n, void *d_ws,
                          size_t bytes, void *hip_stream, float *y_out) {
  try {
    if (!cm || !x || !y_out) return set_err(QTN_EINVAL, "NULL argument");
    int rc = mlp_check_ws(n, d_ws, bytes);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    const MlpBuffers b = mlp_buffers(d_ws, n);
    std::vector<float> stage, y(n * kMlpOut);
    if ((rc = mlp_upload_inputs(cm, x, n, b, true, s, stage))) return rc;
    QTN_HIP(mlp_forward(b, (int)n, s));
    QTN_HIP(hipMemcpyAsync(y.data(), b.y, sizeof(float) * n * kMlpOut, hipMemcpyDeviceToHost, s));
    QTN_HIP(hipStreamSynchronize(s));
    std::copy(y.begin(), y.end(), y_out);
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_costmodel_grad(const qtn_costmodel *cm, const float *x, const float *t, const float *m,
                       int64_t n, void *d_ws, size_t bytes, void *hip_stream, float *loss_out,
                       float *grad_out) {
  try {
    if (!cm || !x || !t || !m || !loss_out || !grad_out) return set_err(QTN_EINVAL, "NULL argument");
    int rc = mlp_check_ws(n, d_ws, bytes);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    const MlpBuffers b = mlp_buffers(d_ws, n);
    std::vector<float> stage, g(kMlpParams);
    if ((rc = mlp_upload_inputs(cm, x, n, b, false, s, stage))) return rc;
    QTN_HIP(hipMemcpyAsync(b.t, t, sizeof(float) * n * kMlpOut, hipMemcpyHostToDevice, s));
    QTN_HIP(hipMemcpyAsync(b.m, m, sizeof(float) * n * kMlpOut, hipMemcpyHostToDevice, s));
    QTN_HIP(mlp_loss_grad(b, (int)n, s));
    float loss = 0;
    QTN_HIP(hipMemcpyAsync(g.data(), b.grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, s));
    QTN_HIP(hipMemcpyAsync(&loss, b.loss, sizeof(float), hipMemcpyDeviceToHost, s));
    QTN_HIP(hipStreamSynchronize(s));
    *loss_out = loss;
    std::copy(g.begin(), g.end(), grad_out);
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_costmodel_adam_step(qtn_costmodel *cm, const float *grad, float lr, void *d_ws,
                            size_t bytes, void *hip_stream) {
  try {
    if (!cm || !grad || !(lr > 0)) return set_err(QTN_EINVAL, "bad arguments");
    int rc = mlp_check_ws(1, d_ws, bytes);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    const MlpBuffers b = mlp_buffers(d_ws, 1);
    QTN_HIP(hipMemcpyAsync(b.params, cm->params.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice, s));
    QTN_HIP(hipMemcpyAsync(b.grad, grad, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, s));
    QTN_HIP(hipMemcpyAsync(b.m1, cm->m1.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice, s));
    QTN_HIP(hipMemcpyAsync(b.m2, cm->m2.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice, s));
    QTN_HIP(mlp_adam(b, cm->step + 1, lr, s));
    std::vector<float> p(kMlpParams), a(kMlpParams), q2(kMlpParams);
    QTN_HIP(hipMemcpyAsync(p.data(), b.params, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, s));
    QTN_HIP(hipMemcpyAsync(a.data(), b.m1, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, s));
    QTN_HIP(hipMemcpyAsync(q2.data(), b.m2, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, s));
    QTN_HIP(hipStreamSynchronize(s));
    cm->params.swap(p);
    cm->m1.swap(a);
    cm->m2.swap(q2);
    cm->step++;
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

int qtn_apply_costmodel(qtn_network *net, const qtn_costmodel *cm, void *d_ws, size_t bytes,
                        void *hip_stream, int32_t *counts_out) {
  try {
    if (!net || !cm) return set_err(QTN_EINVAL, "NULL argument");
    if (!net->planned) return set_err(QTN_ESTATE, "qtn_plan has not been called");
    std::vector<float> feats;
    std::vector<Group *> gs;
    std::vector<const ConePlan *> gp;
    for (ConePlan &pl : net->plans)
      for (Group &G : pl.groups) {
        float f[kNumFeatures];
        group_features(G, pl, net->precision, f);
        feats.insert(feats.end(), f, f + kNumFeatures);
        gs.push_back(&G);
        gp.push_back(&pl);
      }
    const int64_t n = (int64_t)gs.size();
    std::vector<float> y(n * kMlpOut);
    int rc = qtn_costmodel_predict(cm, feats.data(), n, d_ws, bytes, hip_stream, y.data());
    if (rc) return rc;
    int32_t counts[4] = {0, 0, 0, 0};
    for (int64_t i = 0; i < n; i++) {
      Group &G = *gs[i];
      const float *p = &y[i * kMlpOut];
      // placement stays with the width rule: a group's time inside a
      // workgroup segment is not the time of the same group alone in a
      // one-workgroup launch, which is what was measured.  Groups that get
      // their own launch take the kernel with the lowest predicted time, the
      // matrix form only where the group has one.
      G.pick_place = -1;
      if (G.small) {
        G.pick_variant = -1;
        G.pick_rls = -1;
        counts[QTN_VAR_BLOCK]++;
        continue;
      }
      int best = p[QTN_VAR_STREAM] <= p[QTN_VAR_GENERIC] ? QTN_VAR_STREAM : QTN_VAR_GENERIC;
      if (G.prec == 1 && p[QTN_VAR_MFMA] < p[best] && gemm_shape(G, *gp[i], nullptr))
        best = QTN_VAR_MFMA;
      counts[best]++;
      // the streaming family: the cell mapping where it fits, else the
      // lane-sum streaming mapping (the planner falls back by itself)
      G.pick_variant = best == QTN_VAR_STREAM ? 4 : (best == QTN_VAR_MFMA ? 3 : 1);
      G.pick_rls = best == QTN_VAR_STREAM ? kCellRuleCB : 2;
    }
    qtn_network *one[1] = {net};
    auto ex = std::make_unique<Exec>();
    if ((rc = build_schedule(one, 1, &ex->sched, nullptr, 0, 1, net->exec->persistent))) return rc;
    ex->rt.take(net->exec->rt);
    ex->persistent = net->exec->persistent;
    ex->hybrid = net->exec->hybrid;
    ex->dataflow = net->exec->dataflow;
    ex->lead_per_cone = net->exec->lead_per_cone;
    ex->spin_limit = net->exec->spin_limit;
    drop_batches_with(net);
    net->exec = std::move(ex);
    net->version++;
    if (counts_out) std::copy(counts, counts + 4, counts_out);
    return QTN_OK;
  } catch (...) {
    return exception_status();
  }
}

void qtn_costmodel_free(qtn_costmodel *cm) { delete cm; }

void qtn_network_free(qtn_network *net) {
  if (!net) return;
  drop_batches_with(net);
  delete net;
}

}  // extern "C"
