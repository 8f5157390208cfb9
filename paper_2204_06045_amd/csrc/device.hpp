// Device descriptors shared by the host schedule and the HIP kernels.
//
// A fused group (Sec. II-B bucket, or a chain of buckets merged as in
// Sec. II-C) is evaluated over its union index I (w bits, bit 0 = the first
// bucket index eliminated).  Operand t is read at pext(I, mask_t): tensors
// keep their indices sorted by elimination position with the earliest index
// as bit 0, so an operand's layout is the union layout with the absent bits
// squeezed out.  The group sums bits 0..L-1 and writes out[I >> L].
#pragma once

#include <cstdint>

namespace qtn {

constexpr int kOpRuns = 16;

// Operand classes of the streaming mapping (see kernels.hip):
enum OpClass : uint8_t {
  kClsUnit = 0,     // leaf level, no serial bit: constant over a unit's walk
  kClsStep = 1,     // leaf level with serial bits: read at every serial step
  kClsUniform = 2,  // serial level, no lane bit: one table U(s) per unit
  kClsSerial = 3,   // serial level with lane bits: read at every serial step
};

// Angle sets: one launch may evaluate several (gamma, beta) sets on one
// plan; every tensor then has one copy per set, sstride bytes apart.
struct DevOp {          // 64 bytes
  int64_t off;          // byte offset of the operand from the data base (set 0)
  int64_t sstride;      // bytes from one angle set's copy to the next
  uint32_t mask;        // union bits the operand carries
  int32_t stab;         // first entry of its serial-offset table (streaming)
  uint8_t level;        // multiplied in after `level` indices are summed
  uint8_t nruns;        // contiguous runs of `mask`
  uint8_t cls;          // OpClass (streaming)
  uint8_t dt;           // storage: 0 complex128, 1 complex64
  uint16_t run[kOpRuns];  // src | len << 5 | dst << 11 : pext by runs
  uint8_t pad2[4];
};

struct DevGroup {       // 64 bytes
  int64_t out_off;      // byte offset of the output (or scalar slot), set 0
  int64_t out_sstride;  // bytes from one angle set's output to the next
  int32_t op_begin;     // first DevOp of the group
  uint32_t n_units;     // wave units
  uint8_t w, L, n_ops, variant;   // variant: kVar*
  uint8_t rls, sl, lk, n_unit;    // streaming: lane-summed bits, serial bits,
                                  // lane-kept bits, kClsUnit op count
  uint8_t n_step, n_serial, n_step0, pad;  // n_step0: step-class ops with bit 0
  uint8_t level_end[8]; // generic: ops of levels <= l end at level_end[l];
                        // streaming: level_end[0] = uniform-class count; the
                        // n_serial - level_end[0] serial-class ops follow
  uint8_t n_ubits;      // wave-unit bits (their union positions: uperm)
  uint8_t prec;         // arithmetic and output storage: 0 complex128, 1 complex64
  uint8_t cvt;          // 1: some operand is stored in the other precision
  uint8_t n_mb, n_nb, n_bb;  // matrix form: m, n and batch bit counts (their
                             // union positions: uperm, m then n then batch)
  uint8_t lkpos[6];     // streaming: union position of each lane-kept bit
  int32_t gtab;         // matrix form: first entry of the group's row/column table
};

static_assert(sizeof(DevOp) == 64, "DevOp layout");
static_assert(sizeof(DevGroup) == 64, "DevGroup layout");

enum Variant : uint8_t { kVarGeneric = 0, kVarStream = 1, kVarMfma = 2, kVarCell = 3 };

// Cell mapping (kVarCell): lanes are union bits 0..5; rls = cell bits CB held
// in registers per lane: the high sl cell bits are the summed bits 6..L-1
// (serial; cell bit CB - 1 - t is union bit 6 + t), the low CB - sl ones the
// kept bits at union positions uperm[0..CB - sl) (the unit bits follow in
// uperm).  Ops [0, n_step) hold bit 6 (all ops when sl = 0), the next
// n_serial hold bit 7 but not 6 (sl = 2), the rest no serial bit; the first
// n_step0 ops of the last of these levels hold no unit bit (sl = 0: hold lane
// bits only); n_unit = the most unit-bit runs of any operand.  Each op's stab entry starts its table: 2^CB cell offsets
// (elements), kCellURuns / 2 words of unit-bit runs (src | len << 5 | dst <<
// 11, two per word, src counting unit bits; unused runs 0) giving the unit
// part of its index, then the mask of the cell bits its index holds.
constexpr int kCellMinCB = 2, kCellMaxCB = 4, kCellRuleCB = 3;
constexpr int kCellURuns = 16;
constexpr int kCellMaxSerial = 2;
// LDS words of a cell group's tables: per operand 2^CB lane tables of 64
// words and its unit-bit runs.
constexpr int cell_lds_words(int n_ops, int cb) { return n_ops * ((64 << cb) + kCellURuns / 2); }
constexpr int cell_table_words(int cb) { return (1 << cb) + kCellURuns / 2 + 1; }
constexpr int kCellMaxLdsWords = 16384;  // 64 KiB per workgroup

// Matrix form (kVarMfma): ops are [side A..., side B...] with n_unit = |side
// A|, n_step = |side B|.  A work unit is one kMmTM x 16 rls (m x n) output
// tile of one batch index (rls: column blocks, 1, 2 or 4, the most the n
// range fills); a whole workgroup computes it, at most kMmKC summed indices
// per LDS chunk.  Tables (int32, in the stab area): the group's at gtab,
// kMmTM union-bit words for the tile's rows then kMmTN for its columns; each
// operand's at its stab, kMmTM row (side A) or kMmTN column (side B) element
// offsets, then 2^L offsets of the summed indices.
constexpr int kMmTM = 64, kMmTN = 64, kMmKC = 16, kMmMaxOps = 64;

// Generic mapping: 2 register bits and 6 lane bits per wave unit.
constexpr int kGenRegBits = 2;
// Streaming mapping: at most this many operands per group (LDS lane tables).
constexpr int kStreamMaxOps = 96;
constexpr int kStreamMaxSerial = 6;

// Gate table layout (elements; one table per precision in use): per layer l,
// 8 blocks of 4 at 32*l:
// P, P^T, Pc, Pc^T, R, R^T, Rc, Rc^T (row-major over the gate's own axes,
// ^T = the other axis as bit 0); then H (2) at 32*p and Z (2) at 32*p + 2.
inline int64_t gate_table_elems(int p) { return 32LL * p + 4; }

}  // namespace qtn
