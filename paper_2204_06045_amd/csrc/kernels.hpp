// Launchers of the HIP kernels (kernels.hip).  Plain pointers and sizes only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "device.hpp"

namespace qtn {

// Launchers taking (t0, t1): when t0 is not null, the two events are attached
// to the main kernel's dispatch and time that kernel alone.

enum Precision : int { kPrecC128 = 0, kPrecC64 = 1, kPrecMixed = 2 };

// One block per network: fills that network's gate table from its angles.
struct FillDesc {
  int64_t angle_off;  // doubles from an angle set's base: gamma[p] then beta[p]
  int64_t table128;   // byte offset of the complex128 gate table (set 0), or -1
  int64_t table64;    // byte offset of the complex64 gate table (set 0), or -1
  int64_t sstride128, sstride64;  // bytes between angle sets' tables
  int32_t p, pad;
};

// n_sets angle sets of n_angles doubles each, set after set.
hipError_t launch_fill(int prec, void *data, const double *angles,
                       const FillDesc *fills, int n_nets, int n_angles, int n_sets,
                       hipStream_t s);

// Groups [ranges[b].x, ranges[b].y) run in order inside one block, for
// b in [range_base, range_base + n_blocks), once per angle set (n_blocks *
// n_sets blocks).  uperm holds 32 bytes per group: the union bit of each
// wave-unit bit.
hipError_t launch_block_groups(int prec, void *data, const DevGroup *groups,
                               const DevOp *ops, const int32_t *stab,
                               const uint8_t *uperm, const int2 *ranges,
                               int range_base, int n_blocks, int n_sets, hipStream_t s,
                               hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);

// One group over the whole grid, with the kernel of its mapping variant and
// precision; hg is the host copy of the group's descriptor.
hipError_t launch_wide_group(const DevGroup &hg, void *data, const DevGroup *groups,
                             const DevOp *ops, const int32_t *stab, const uint8_t *uperm,
                             int group, int n_sets, hipStream_t s, hipEvent_t t0 = nullptr,
                             hipEvent_t t1 = nullptr);

// Clears the control words, then runs every light cone's task list in
// lockstep inside one persistent launch of n_blocks resident blocks.
// items: (group_begin, group_end, 0, 0) for a segment of small groups or
// (group, -1, unit_begin, unit_end) for a chunk of a wide group; step s owns
// items [step_begin[s], step_begin[s+1]).  ctl needs 4 + n_steps words;
// ctl[2] != 0 after the launch means a barrier wait exceeded spin_limit.
hipError_t launch_persistent(int prec, void *data, const DevGroup *groups,
                             const DevOp *ops, const int32_t *stab,
                             const uint8_t *uperm, const int4 *items, const int *step_begin, int n_steps,
                             uint32_t *ctl, int n_ctl, int n_blocks,
                             uint32_t spin_limit, hipStream_t s, hipEvent_t t0 = nullptr,
                             hipEvent_t t1 = nullptr);

// Runs every cone's tasks inside one persistent launch with a ready queue:
// items of task t are items[task_first[t] .. task_first[t] + task_need[t]);
// task_next[t] is the next task of the same light cone (-1: none); the first
// n_init items (the first task of every cone) are ready at the start.  A
// task's successor is queued when the task's last item completes.  queue
// holds n_items words; ctl needs 4 + n_tasks words (ctl[2] != 0 after the
// launch means a wait exceeded spin_limit).
hipError_t launch_dataflow(void *data, const DevGroup *groups, const DevOp *ops,
                           const int32_t *stab, const uint8_t *uperm, const int4 *items,
                           int n_items, int n_init, const int *item_task, const int *task_next,
                           const int *task_first, const int *task_need, uint32_t *queue,
                           uint32_t *ctl, int n_ctl, int n_blocks, uint32_t spin_limit,
                           hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);

// Resident blocks of the persistent kernel on n_cu compute units (0 on error).
int persistent_blocks(int prec, int n_cu);

// All offsets in descriptors are bytes from the data base `data`.
// launch_reduce: scalars stored as complex64 when prec is kPrecC64, else as
// complex128, starting scalar_off bytes into data.
// Per light cone: product of its scalar slots -> e_jk (FP64); with index
// slicing (cone_slices[c] > 1) the slots split into that many equal runs, one
// per slice, and e_jk is the sum of the runs' products; per network:
// E = |E|/2 - 1/2 sum Re e_jk with Neumaier compensation.
// res: per angle set [n_cones] Re, [n_cones] Im, [n_nets] energies.
hipError_t launch_reduce(int prec, const void *data, int64_t scalar_off,
                         int64_t scalar_sstride, const int *cone_scalar_begin,
                         const int *net_cone_begin, const int *cone_slices, int n_cones,
                         int n_nets, int n_sets, double *res, hipStream_t s);


// Bytes of the device scratch array that the allocation-free bucket entry
// point copies its descriptors into.
constexpr size_t kScratchBytes = 16384;

// Device address of that array on the current device (looked up once per
// device with hipGetSymbolAddress; never the host-side name).
hipError_t scratch_address(void **out);

}  // namespace qtn
