// Host-side planner: light cones, tensor networks, elimination orders,
// symbolic bucket elimination, merged-index groups and the memory plan.
//
// Method references (arXiv 2204.06045):
//   Sec. II-A, Eq. 1-2   QAOA MaxCut ansatz and cost operator
//   Sec. II-B            light cones, circuit -> tensor network, buckets,
//                        bucket width, energy as a sum of edge terms
//   Sec. II-C            merged indices: buckets whose index sets nest are
//                        summed together in one pass
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace qtn {

constexpr int kMaxWidth = 32;     // union index of a group fits in 32 bits
constexpr int kMaxLevels = 8;     // summed indices per fused group
constexpr int kMaxRuns = 16;      // contiguous bit runs of an operand mask

enum GateKind : int8_t { kH = 0, kZ = 1, kP = 2, kPc = 3, kR = 4, kRc = 5 };

// One gate tensor.  Its value table is row-major over (var[0], var[1]):
//   H  = (1, 1)/sqrt2                     rank 1, |+> amplitude
//   Z  = (1, -1)                          rank 1, observable factor
//   P  = exp(-i gamma [x0 != x1])         rank 2, cost phase (Eq. 1)
//   R  = <x0| exp(-i beta X) |x1>         rank 2, mixer (Eq. 2)
//   Pc, Rc = complex conjugates (bra side)
struct Gate {
  GateKind kind;
  int8_t layer;  // 0-based QAOA layer of P/Pc/R/Rc
  int8_t rank;
  int32_t var[2];
  // Index slicing: a rank-2 gate one of whose variables is fixed.  `cut` is
  // the fixed axis of the original gate (0 or 1); the gate is then stored as
  // rank 1 over the other variable (var[0]), and the fixed value is bit
  // `cut_slot` of the slice number.  -1: not cut.
  int8_t cut = -1;
  int8_t cut_slot = -1;
};

struct LightCone {
  int edge = -1, j = -1, k = -1;
  int n_vars = 0;
  std::vector<Gate> gates;
};

struct Graph {
  int n = 0;
  std::vector<int> eu, ev;   // edge endpoints
  std::vector<std::vector<int>> adj;
};

// Validates and stores a graph; returns an error message or "".
std::string make_graph(int n, int64_t m, const int32_t *edges, Graph *g);

// Light cone of edge e at depth p (Sec. II-B reverse light cone).
LightCone build_lightcone(const Graph &g, int e, int p);

struct PlanOptions;

// Greedy min-fill order (ties: fewest neighbours, then smallest id; with a
// nonzero seed, remaining ties are broken at random).
std::vector<int> minfill_order(const LightCone &lc, uint64_t seed = 0);

// Sum over buckets of 2^width for an order (index sets only).
double order_cost(const LightCone &lc, const std::vector<int> &order);

// Width of the widest bucket for an order; `widest` (optional) receives the
// variables of that bucket's union.
int order_width(const LightCone &lc, const std::vector<int> &order,
                std::vector<int> *widest = nullptr);

// Index slicing (the network's scalar is the sum, over the 2^s values of s
// fixed variables, of the scalars of the networks with those variables
// fixed): the light cone with variable `var` fixed, as slice bit `slot`.
// Every gate holding `var` must be rank 2; it becomes rank 1 (Gate::cut).
LightCone slice_cone(const LightCone &lc, int var, int slot);

// Variables to fix so that the widest bucket is at most `cap`: greedily,
// the variable of the current widest bucket whose fixing gives the
// narrowest (then cheapest) min-fill plan, at most `max_vars` of them.
// Only variables held by rank-2 gates alone, and sharing no gate with an
// already fixed one, are fixed (so every gate keeps an index).  Returns the
// variables in slot order and, in order_out, the order of the restricted
// light cone that reached the last width; the caller checks that width.
std::vector<int> choose_slices(const LightCone &lc, int cap, int max_vars, int trials,
                               std::vector<int> *order_out = nullptr,
                               const PlanOptions *plan = nullptr, double bytes_weight = 0);

// The cheapest of the greedy order and trials-1 randomized min-fill orders:
// by order_cost (sum of 2^width), or, with `plan` given, by the merged plan's
// complex flops + bytes_weight * algorithmic bytes (the groups the kernels
// actually run, under those plan options).
std::vector<int> search_order(const LightCone &lc, int trials, const PlanOptions *plan = nullptr,
                              double bytes_weight = 0);

// ---------------------------------------------------------------- plan

struct Tensor {
  std::vector<int> vars;   // sorted by elimination position (bit 0 first)
  int gate = -1;           // initial tensor: index into LightCone::gates
  bool transposed = false; // rank-2 gate stored with var[0] as bit 0
  int producer = -1;       // group writing this intermediate
  int consumer = -1;       // group reading it
  int64_t offset = -1;     // byte offset inside the light cone's arena
  int8_t prec = 0;         // storage: 0 complex128, 1 complex64
};

struct Operand {
  int tensor;
  uint32_t mask;  // union bits the operand carries
  int level;      // 0..L-1: multiplied in after that many indices are summed
};

struct Group {
  int w = 0;                 // union width
  int L = 0;                 // bucket indices summed (merged buckets)
  int first_pos = 0, last_pos = 0; // elimination positions of the members
  std::vector<Operand> ops;  // sorted by level
  int out_tensor = -1;       // -1: scalar output
  int scalar_slot = -1;      // light cone's scalar slot when out_tensor < 0
  bool small = false;        // runs inside one workgroup
  int8_t prec = 0;           // arithmetic: 0 complex128, 1 complex64
  // kernel choice from the autotuner or the cost model (-1: width rule)
  int8_t pick_place = -1;    // 0 inside a workgroup segment, 1 own launch
  int8_t pick_variant = -1;  // 1 generic mapping, 2 streaming mapping
  int8_t pick_rls = -1;      // streaming: lane-summed bits
};


struct ConePlan {
  // index slicing: the plan is of the light cone with slice_vars fixed; its
  // groups run once per slice (n_slices = 2^|slice_vars|) and the cone's
  // scalar is the sum of the slices' scalars.  gates: that light cone's gates
  // (empty when nothing is sliced: the original cone's gates apply)
  std::vector<int> slice_vars;
  int n_slices = 1;
  std::vector<Gate> gates;
  std::vector<int> order;
  std::vector<int> bucket_width;   // by elimination position, 0 if empty
  int max_width = 0;
  int n_buckets = 0;
  std::vector<Tensor> tensors;
  std::vector<Group> groups;       // in execution order
  int n_scalars = 0;
  int64_t arena_bytes = 0;         // peak live bytes of intermediates
  double bytes = 0, flops = 0, paper_flops = 0;  // per evaluation
};

// Matrix form of a group.  The merged contraction of Sec. II-C is a batched
// complex matrix product once the group's operands are split into two sides:
//   out[bt, m, n] = sum_k At[bt, m, k] Bt[bt, k, n]
// At (Bt) is the product of the side-A (side-B) operands; k runs over the L
// summed union bits (0..L-1); m over kept bits held on side A only, n over
// kept bits held on side B only, bt over kept bits held on both.  Every split
// is exact; the matrix cores pay off when m and n are both wide, so the split
// keeps each side's private kept bits many.
struct GemmShape {
  int a = -1, b = -1;            // the two operands the sides are built around
  std::vector<int8_t> role;      // per operand: 0 side A, 1 side B
  std::vector<int> mbits, nbits, bbits;  // union bit positions, low to high
};

// The matrix form of G, or false when G has none worth running: fewer than
// two operands, more than 64, or fewer than 4 n bits (one 16-wide block of
// the matrix cores).  Side A is built around the largest operand, side B
// around the one with the most kept bits side A lacks; |m| >= |n|.
bool gemm_shape(const Group &G, const ConePlan &pl, GemmShape *gs);

// 16 shape features of a group, for timing records and the cost model.
constexpr int kNumFeatures = 16;
void group_features(const Group &G, const ConePlan &pl, int precision, float *f);

constexpr int kMaxSliceVars = 10;  // at most 1024 slices per light cone

struct PlanOptions {
  int slice_width = 0;   // >0: fix variables of light cones wider than this
  int order_weight = 0;  // >0: order search by plan flops + order_weight * bytes
  int max_levels = kMaxLevels;
  int small_width = 12;
  int max_width = kMaxWidth;
  int precision = 0;     // 0 complex128, 1 complex64, 2 mixed
  int mixed_width = 18;  // mixed: groups at least this wide run in complex64
};

// Symbolic bucket elimination of one light cone along `order`, merged into
// groups, with the arena laid out.  Returns an error message or "".
std::string plan_cone(const LightCone &lc, const std::vector<int> &order,
                      const PlanOptions &opt, ConePlan *out);

// Bit runs of a mask: pext(x, mask) = sum over runs of
// ((x >> src) & ((1 << len) - 1)) << dst.
int mask_runs(uint32_t mask, uint8_t *src, uint8_t *len, uint8_t *dst);

}  // namespace qtn
