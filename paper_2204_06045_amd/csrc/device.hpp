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

struct DevOp {          // 64 bytes
  int64_t off;          // element offset of the operand from the data base
  uint32_t mask;        // union bits the operand carries
  uint8_t level;        // multiplied in after `level` indices are summed
  uint8_t nruns;        // contiguous runs of `mask`
  uint8_t pad[2];
  uint8_t rs[16];       // run start bit in I
  uint8_t rl[16];       // run length
  uint8_t rd[16];       // run start bit in the operand offset
};

struct DevGroup {       // 32 bytes
  int64_t out_off;      // element offset of the output (or scalar slot)
  int32_t op_begin;     // first DevOp of the group
  uint32_t n_units;     // wave units: 2^max(0, w - units_shift)
  uint8_t w, L, n_ops, pad;
  uint8_t level_end[8]; // ops of levels 0..l end at op_begin + level_end[l]
  uint8_t pad2[4];
};

static_assert(sizeof(DevOp) == 64, "DevOp layout");
static_assert(sizeof(DevGroup) == 32, "DevGroup layout");

// Gate table layout (elements): per layer l, 8 blocks of 4 at 32*l:
// P, P^T, Pc, Pc^T, R, R^T, Rc, Rc^T (row-major over the gate's own axes,
// ^T = the other axis as bit 0); then H (2) at 32*p and Z (2) at 32*p + 2.
inline int64_t gate_table_elems(int p) { return 32LL * p + 4; }

}  // namespace qtn
