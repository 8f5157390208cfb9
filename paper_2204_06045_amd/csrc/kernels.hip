// HIP kernels for gfx950 (CDNA4): bucket contraction over fused groups.
//
// Bucket elimination (arXiv 2204.06045, Sec. II-B) contracts a bucket by
// multiplying its tensors over the union of their binary indices and summing
// the bucket index; merged indices (Sec. II-C) sum several nested buckets in
// one pass.  A fused group is such a chain of L buckets over the union index I
// (bit 0 = first bucket index): level-l operands are multiplied in after bits
// 0..l-1 are summed, and the group writes out[I >> L].  Every operand t is
// read at pext(I, mask_t).
//
// Two thread mappings (wave64):
//
// Streaming (kVarStream).  Bit 0 lives in registers (two points per lane);
// the next `rls` summed bits select lanes (contiguous operand runs per lane
// group, summed at the end with cross-lane butterflies); the remaining `sl`
// summed bits are walked serially by each lane; the kept bits select the
// other `lk` lanes and the wave unit.  Operand offsets split into a lane part
// (pext of the lane bits, staged once per group in LDS), a unit part (pext of
// the unit bits, wave-uniform, scalar ALU) and a serial part (per-step table
// built by the planner), so the inner loop is loads and complex FMAs.  The
// group's sum is taken flat: a level-l operand does not depend on bits 0..l-1,
// so multiplying it in before those bits are summed gives the same sum; the
// nesting only decides how often each factor is applied.
//
// Generic (kVarGeneric).  2 register bits and 6 lane bits per unit, every
// level in hierarchical order with register adds and lane butterflies.  Used
// for groups with more operands than the streaming LDS tables hold.
//
// Matrix form (kVarMfma).  A group whose operands split into two sides is a
// batched complex matrix product of the sides' factors; it runs as three real
// products on the matrix cores (3M), FP32 for complex64 and FP64 for
// complex128 groups.
#include <cstddef>
#include <map>
#include <mutex>
#include <tuple>

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace qtn {
namespace {

constexpr int kBlock = 256;
constexpr int kStepOps = 4;  // step-class operands unrolled in the serial loop
constexpr int kGenBatch = 3; // generic mapping: leaf operands loaded together

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 shfl_xor2(double2 v, int m) {
  return make_double2(__shfl_xor(v.x, m), __shfl_xor(v.y, m));
}
__device__ __forceinline__ float2 shfl_xor2(float2 v, int m) {
  return make_float2(__shfl_xor(v.x, m), __shfl_xor(v.y, m));
}
template <class T> __device__ __forceinline__ T make_c(double re, double im);
template <> __device__ __forceinline__ double2 make_c<double2>(double re, double im) {
  return make_double2(re, im);
}
template <> __device__ __forceinline__ float2 make_c<float2>(double re, double im) {
  return make_float2((float)re, (float)im);
}
__device__ __forceinline__ double2 to_d(double2 v) { return v; }
__device__ __forceinline__ double2 to_d(float2 v) { return make_double2(v.x, v.y); }

// Element storage: dt 0 = complex128 (double2), 1 = complex64 (float2).  With
// CVT false every operand of the group is stored as T and dt is not read.
template <class T, bool CVT> __device__ __forceinline__ uint32_t esize(int dt) {
  return CVT ? (dt ? 8u : 16u) : (uint32_t)sizeof(T);
}

// Element `idx` of an operand stored as dt at p, converted to T.
template <class T, bool CVT> __device__ __forceinline__ T ld_elem(const char *p, uint64_t idx, int dt);
template <> __device__ __forceinline__ double2 ld_elem<double2, false>(const char *p, uint64_t idx, int) {
  return *(const double2 *)(p + idx * 16u);
}
template <> __device__ __forceinline__ float2 ld_elem<float2, false>(const char *p, uint64_t idx, int) {
  return *(const float2 *)(p + idx * 8u);
}
template <> __device__ __forceinline__ double2 ld_elem<double2, true>(const char *p, uint64_t idx, int dt) {
  if (dt == 0) return *(const double2 *)(p + idx * 16u);
  const float2 v = *(const float2 *)(p + idx * 8u);
  return make_double2(v.x, v.y);
}
template <> __device__ __forceinline__ float2 ld_elem<float2, true>(const char *p, uint64_t idx, int dt) {
  if (dt == 1) return *(const float2 *)(p + idx * 8u);
  const double2 v = *(const double2 *)(p + idx * 16u);
  return make_float2((float)v.x, (float)v.y);
}

// Descriptor fields are read as 32-bit words: at wave-uniform addresses these
// become scalar loads, while sub-dword fields would be vector loads on the
// critical path of every operand.
__device__ __forceinline__ uint32_t dword(const void *p, int i) {
  return reinterpret_cast<const uint32_t *>(p)[i];
}
static_assert(offsetof(DevOp, level) == 24 && offsetof(DevOp, dt) == 27 &&
                  offsetof(DevOp, run) == 28,
              "DevOp word layout");
__device__ __forceinline__ int op_nruns(const DevOp &o) { return (dword(&o, 6) >> 8) & 0xFFu; }
__device__ __forceinline__ int op_dt(const DevOp &o) { return dword(&o, 6) >> 24; }
__device__ __forceinline__ uint32_t op_run(const DevOp &o, int i) {
  return (dword(&o, 7 + (i >> 1)) >> ((i & 1) * 16)) & 0xFFFFu;
}
// Union position of wave-unit bit j from a group's 32-byte unit-bit table.
__device__ __forceinline__ uint32_t ubit_at(const uint8_t *ub, int j) {
  return (dword(ub, j >> 2) >> ((j & 3) * 8)) & 0xFFu;
}

// A group's header unpacked from its descriptor words (wave-uniform values).
struct GI {
  int64_t out_off, out_sstride;
  uint32_t op_begin, n_units;
  int w, L, n_ops, variant, rls, sl, lk, n_unit, n_step, n_serial, n_step0;
  int n_ubits, prec, cvt, n_mb, n_nb, n_bb;
  int32_t gtab;           // matrix form: the group's row and column table
  uint32_t le_lo, le_hi;  // level_end[0..3], [4..7]
  uint32_t lk_lo, lk_hi;  // lkpos[0..1], [2..5]
  __device__ int le(int l) const { return ((l < 4 ? le_lo >> (8 * l) : le_hi >> (8 * (l - 4)))) & 0xFF; }
  // union bits of the lane-kept part of a lane (streaming mapping)
  __device__ uint32_t lane_kept(uint32_t hi) const {
    uint32_t I = 0;
    for (int j = 0; j < lk; j++) {
      const uint32_t pos = (j < 2 ? lk_lo >> (8 * j) : lk_hi >> (8 * (j - 2))) & 0xFFu;
      I |= ((hi >> j) & 1u) << pos;
    }
    return I;
  }
};
static_assert(offsetof(DevGroup, w) == 24 && offsetof(DevGroup, rls) == 28 &&
                  offsetof(DevGroup, n_step) == 32 && offsetof(DevGroup, level_end) == 36 &&
                  offsetof(DevGroup, n_ubits) == 44 && offsetof(DevGroup, n_nb) == 48 &&
                  offsetof(DevGroup, lkpos) == 50 && offsetof(DevGroup, gtab) == 56,
              "DevGroup word layout");
__device__ __forceinline__ GI load_group(const DevGroup *g) {
  GI G;
  const uint32_t w0 = dword(g, 0), w1 = dword(g, 1), w2 = dword(g, 2), w3 = dword(g, 3);
  G.out_off = (int64_t)(((uint64_t)w1 << 32) | w0);
  G.out_sstride = (int64_t)(((uint64_t)w3 << 32) | w2);
  G.op_begin = dword(g, 4);
  G.n_units = dword(g, 5);
  const uint32_t a = dword(g, 6), b = dword(g, 7), c = dword(g, 8), e = dword(g, 11),
                 f = dword(g, 12);
  G.w = a & 0xFF;
  G.L = (a >> 8) & 0xFF;
  G.n_ops = (a >> 16) & 0xFF;
  G.variant = a >> 24;
  G.rls = b & 0xFF;
  G.sl = (b >> 8) & 0xFF;
  G.lk = (b >> 16) & 0xFF;
  G.n_unit = b >> 24;
  G.n_step = c & 0xFF;
  G.n_serial = (c >> 8) & 0xFF;
  G.n_step0 = (c >> 16) & 0xFF;
  G.le_lo = dword(g, 9);
  G.le_hi = dword(g, 10);
  G.n_ubits = e & 0xFF;
  G.prec = (e >> 8) & 0xFF;
  G.cvt = (e >> 16) & 0xFF;
  G.n_mb = e >> 24;
  G.n_nb = f & 0xFF;
  G.n_bb = (f >> 8) & 0xFF;
  G.lk_lo = f >> 16;
  G.lk_hi = dword(g, 13);
  G.gtab = (int32_t)dword(g, 14);
  return G;
}

// pext(x, mask) from the operand's packed runs (wave-uniform loop bounds).
__device__ __forceinline__ uint32_t pext_runs(uint32_t x, const DevOp &o) {
  uint32_t r = 0;
  const int nr = op_nruns(o);
  for (int i = 0; i < nr; i++) {
    const uint32_t rr = op_run(o, i);
    const uint32_t src = rr & 31u, len = (rr >> 5) & 63u, dst = rr >> 11;
    r |= ((x >> src) & (uint32_t)((1ull << len) - 1ull)) << dst;
  }
  return r;
}

// Operand and output of angle set `set` (each tensor has one copy per set).
__device__ __forceinline__ const char *opnd(const char *data, const DevOp &o, uint32_t set) {
  return data + o.off + (int64_t)set * o.sstride;
}
__device__ __forceinline__ char *outp(char *data, const GI &G, uint32_t set) {
  return data + G.out_off + (int64_t)set * G.out_sstride;
}

// Union bits of wave unit u: bit j of u goes to union bit ubit[j] (the
// planner orders the unit bits so that bits some large operand lacks come
// first, and units that reuse an operand's data run next to each other).
__device__ __forceinline__ uint32_t unit_bits(uint32_t u, const uint8_t *__restrict__ ubit,
                                              int n, int first = 0) {
  // ubit is a group's 4-byte aligned table; bits first..first+n-1 are used
  uint32_t I = 0;
  for (int j = 0; j < n; j++) I |= ((u >> j) & 1u) << ubit_at(ubit, first + j);
  return I;
}

// ------------------------------------------------------------------ generic

__device__ __forceinline__ uint32_t pext_reg(uint32_t x, uint32_t m) {
  uint32_t r = 0, d = 0;
#pragma unroll
  for (int b = 0; b < kGenRegBits; b++)
    if ((m >> b) & 1u) {
      r |= ((x >> b) & 1u) << d;
      d++;
    }
  return r;
}

template <class T, bool CVT>
__device__ __forceinline__ void generic_unit(const GI &G, const DevOp *__restrict__ gops,
                                             const uint8_t *__restrict__ ubit, char *__restrict__ data,
                                             uint32_t u, int lane, uint32_t set) {
  constexpr int RG = kGenRegBits, NR = 1 << RG;
  const uint32_t I0 = unit_bits(u, ubit, G.n_ubits) | ((uint32_t)lane << RG);
  const int L = G.L;
  T v[NR];
  {
    const DevOp &o = gops[0];
    const uint32_t base = pext_runs(I0, o);
    const char *src = opnd(data, o, set);
#pragma unroll
    for (int r = 0; r < NR; r++) v[r] = ld_elem<T, CVT>(src, base + pext_reg(r, o.mask), op_dt(o));
  }
  // the other leaf operands, kGenBatch at a time: all of their loads are
  // issued before the first multiply, so their latencies overlap
  int k = 1;
  const int e0 = G.le(0);
  for (; k + kGenBatch <= e0; k += kGenBatch) {
    T x[kGenBatch][NR];
#pragma unroll
    for (int j = 0; j < kGenBatch; j++) {
      const DevOp &o = gops[k + j];
      const uint32_t base = pext_runs(I0, o);
      const char *src = opnd(data, o, set);
#pragma unroll
      for (int r = 0; r < NR; r++) x[j][r] = ld_elem<T, CVT>(src, base + pext_reg(r, o.mask), op_dt(o));
    }
#pragma unroll
    for (int j = 0; j < kGenBatch; j++)
#pragma unroll
      for (int r = 0; r < NR; r++) v[r] = cmul(v[r], x[j][r]);
  }
  for (; k < e0; k++) {
    const DevOp &o = gops[k];
    const uint32_t base = pext_runs(I0, o);
    const char *src = opnd(data, o, set);
#pragma unroll
    for (int r = 0; r < NR; r++)
      v[r] = cmul(v[r], ld_elem<T, CVT>(src, base + pext_reg(r, o.mask), op_dt(o)));
  }
#pragma unroll
  for (int s = 0; s < RG; s++) {
    if (s < L) {
#pragma unroll
      for (int r = 0; r < (NR >> (s + 1)); r++) v[r] = cadd(v[2 * r], v[2 * r + 1]);
      if (s + 1 < L) {
        for (; k < G.le(s + 1); k++) {
          const DevOp &o = gops[k];
          const uint32_t base = pext_runs(I0, o);
          const char *src = opnd(data, o, set);
#pragma unroll
          for (int r = 0; r < (NR >> (s + 1)); r++)
            v[r] = cmul(v[r], ld_elem<T, CVT>(src, base + pext_reg((uint32_t)r << (s + 1), o.mask), op_dt(o)));
        }
      }
    }
  }
  T *out = (T *)outp(data, G, set);
  const uint32_t nout = 1u << (G.w - L);
  if (L <= RG) {
    const uint32_t ob = I0 >> L;
#pragma unroll
    for (int r = 0; r < NR; r++)
      if (r < (NR >> L) && ob + r < nout) out[ob + r] = v[r];
    return;
  }
  T acc = v[0];
  for (int s = RG; s < L; s++) {
    acc = cadd(acc, shfl_xor2(acc, 1 << (s - RG)));
    if (s + 1 < L) {
      for (; k < G.le(s + 1); k++) {
        const DevOp &o = gops[k];
        acc = cmul(acc, ld_elem<T, CVT>(opnd(data, o, set), pext_runs(I0, o), op_dt(o)));
      }
    }
  }
  if ((lane & ((1 << (L - RG)) - 1)) == 0) {
    const uint32_t o = I0 >> L;
    if (o < nout) out[o] = acc;
  }
}

// ---------------------------------------------------------------- streaming

// Lane parts of every operand of the group: pext of the lane bits.
__device__ __forceinline__ void stream_setup(const GI &G, const DevOp *__restrict__ gops,
                                             uint32_t *s_lane) {
  const uint32_t rls = G.rls;
  for (int e = threadIdx.x; e < G.n_ops * 64; e += blockDim.x) {
    const int k = e >> 6, lane = e & 63;
    const uint32_t lo = (uint32_t)lane & ((1u << rls) - 1u), hi = (uint32_t)lane >> rls;
    s_lane[e] = pext_runs((lo << 1) | G.lane_kept(hi), gops[k]);
  }
}

__device__ __forceinline__ double2 readlane2(double2 v, uint32_t l) {
  const int2 a = make_int2(__builtin_amdgcn_readlane(__double2loint(v.x), l),
                           __builtin_amdgcn_readlane(__double2hiint(v.x), l));
  const int2 b = make_int2(__builtin_amdgcn_readlane(__double2loint(v.y), l),
                           __builtin_amdgcn_readlane(__double2hiint(v.y), l));
  return make_double2(__hiloint2double(a.y, a.x), __hiloint2double(b.y, b.x));
}
__device__ __forceinline__ float2 readlane2(float2 v, uint32_t l) {
  return make_float2(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.x), l)),
                     __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.y), l)));
}

// A wave-uniform pointer, forced into scalar registers.
__device__ __forceinline__ const char *uniform_ptr(const void *p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (const char *)(((uint64_t)hi << 32) | lo);
}

// Global load at (scalar base + per-lane byte offset), through a global
// address-space pointer so the compiler emits global (not flat) loads.
typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf2 __attribute__((ext_vector_type(2)));
template <class T> __device__ __forceinline__ T gload(const char *base, uint32_t byte_off);
template <> __device__ __forceinline__ double2 gload<double2>(const char *base, uint32_t byte_off) {
  typedef const char __attribute__((address_space(1))) gchar;
  typedef const nd2 __attribute__((address_space(1))) gv;
  const nd2 v = *(gv *)((gchar *)base + byte_off);
  return make_double2(v.x, v.y);
}
template <> __device__ __forceinline__ float2 gload<float2>(const char *base, uint32_t byte_off) {
  typedef const char __attribute__((address_space(1))) gchar;
  typedef const nf2 __attribute__((address_space(1))) gv;
  const nf2 v = *(gv *)((gchar *)base + byte_off);
  return make_float2(v.x, v.y);
}

// The same with the operand stored as dt (CVT) or as T, converted to T.
template <class T, bool CVT>
__device__ __forceinline__ T gload_dt(const char *base, uint32_t off, int dt) {
  if (!CVT) return gload<T>(base, off);
  if (dt == (sizeof(T) == 16 ? 0 : 1)) return gload<T>(base, off);
  if (sizeof(T) == 16) {
    const float2 v = gload<float2>(base, off);
    return make_c<T>(v.x, v.y);
  }
  const double2 v = gload<double2>(base, off);
  return make_c<T>(v.x, v.y);
}

// One wave unit of the streaming mapping.  With u fixed, every point's value
// is the product of
//   unit-class operands      (no serial bit)        -> c0, c1 once per unit
//   step-class operands      (leaf level, serial bits) -> loaded each step
//   uniform-class operands   (serial level, no lane bit) -> table U(s), one
//                            entry per lane, built once per unit
//   serial-class operands    (serial level, lane bits)  -> loaded each step
// summed over bit 0 (registers), the serial bits (this loop) and the
// lane-summed bits (butterflies).  Operands without bit 0 multiply the pair
// sum once instead of each point.  Serial offsets of the unrolled operands sit
// one entry per lane and are read with readlane, so a step's loads issue
// back to back from scalar bases.
template <class T, bool CVT>
__device__ __forceinline__ void stream_unit(const GI &G, const DevOp *__restrict__ gops,
                                            const int32_t *__restrict__ stab,
                                            const uint8_t *__restrict__ ubit, char *__restrict__ data,
                                            const uint32_t *s_lane, uint32_t u, int lane,
                                            uint32_t set) {
  const int L = G.L, rls = G.rls, sl = G.sl;
  const uint32_t Iu = unit_bits(u, ubit, G.n_ubits);
  const uint32_t nsteps = 1u << sl;
  const bool lane_step = (uint32_t)lane < nsteps;
  const T one = make_c<T>(1.0, 0.0);
  T c0 = one, c1 = one;
  for (int k = 0; k < G.n_unit; k++) {
    const DevOp &o = gops[k];
    const uint32_t ES = esize<T, CVT>(op_dt(o));
    const char *p = uniform_ptr(opnd(data, o, set) + (uint64_t)pext_runs(Iu, o) * ES);
    const uint32_t lb = s_lane[k * 64 + lane] * ES;
    const T x0 = gload_dt<T, CVT>(p, lb, op_dt(o));
    const T x1 = gload_dt<T, CVT>(p, lb + ((o.mask & 1u) ? ES : 0u), op_dt(o));
    c0 = cmul(c0, x0);
    c1 = cmul(c1, x1);
  }
  // U(s) for s = lane: product of the uniform-class operands at step s
  const int ku = G.n_unit + G.n_step, ks = ku + G.le(0);
  T U = one;
  for (int k = ku; k < ks; k++) {
    const DevOp &o = gops[k];
    const uint32_t ES = esize<T, CVT>(op_dt(o));
    const char *p = uniform_ptr(opnd(data, o, set) + (uint64_t)pext_runs(Iu, o) * ES);
    const uint32_t off = lane_step ? (uint32_t)stab[o.stab + lane] * ES : 0u;
    U = cmul(U, gload_dt<T, CVT>(p, off, op_dt(o)));
  }
  // unrolled step-class operands: scalar base, per-lane byte offset, serial
  // offsets one per lane
  const int kb = G.n_unit, n_step = G.n_step;
  const char *pb[kStepOps];
  uint32_t lb[kStepOps], tb[kStepOps], h0b[kStepOps];
  bool h0[kStepOps];
  int dt[kStepOps];
#pragma unroll
  for (int i = 0; i < kStepOps; i++) {
    pb[i] = uniform_ptr(data);
    lb[i] = 0;
    tb[i] = 0;
    h0[i] = false;
    h0b[i] = 0;
    dt[i] = 0;
    if (i < n_step) {
      const DevOp &o = gops[kb + i];
      const uint32_t ES = esize<T, CVT>(op_dt(o));
      dt[i] = op_dt(o);
      pb[i] = uniform_ptr(opnd(data, o, set) + (uint64_t)pext_runs(Iu, o) * ES);
      lb[i] = s_lane[(kb + i) * 64 + lane] * ES;
      tb[i] = lane_step ? (uint32_t)stab[o.stab + lane] * ES : 0u;
      h0[i] = (o.mask & 1u) != 0;
      h0b[i] = h0[i] ? ES : 0u;
    }
  }
  const int ke = ks + G.n_serial - G.le(0);  // end of serial-class ops
  T acc = make_c<T>(0.0, 0.0);
  for (uint32_t s = 0; s < nsteps; s++) {
    T e0[kStepOps], e1[kStepOps];
#pragma unroll
    for (int i = 0; i < kStepOps; i++) {
      e0[i] = one;
      e1[i] = one;
      if (i < n_step) {
        const char *p = pb[i] + __builtin_amdgcn_readlane(tb[i], s);
        e0[i] = gload_dt<T, CVT>(p, lb[i], dt[i]);
        e1[i] = gload_dt<T, CVT>(p, lb[i] + h0b[i], dt[i]);
      }
    }
    T v0 = c0, v1 = c1;
#pragma unroll
    for (int i = 0; i < kStepOps; i++)
      if (i < n_step && h0[i]) {
        v0 = cmul(v0, e0[i]);
        v1 = cmul(v1, e1[i]);
      }
    // step operands past the unrolled slots: those with bit 0 come first
    const int k_extra = kb + kStepOps, k_h0_end = kb + G.n_step0;
    for (int k = k_extra; k < k_h0_end; k++) {
      const DevOp &o = gops[k];
      const uint32_t ES = esize<T, CVT>(op_dt(o));
      const char *p = uniform_ptr(opnd(data, o, set) +
                                  ((uint64_t)pext_runs(Iu, o) + (uint32_t)stab[o.stab + s]) * ES);
      const uint32_t l = s_lane[k * 64 + lane] * ES;
      v0 = cmul(v0, gload_dt<T, CVT>(p, l, op_dt(o)));
      v1 = cmul(v1, gload_dt<T, CVT>(p, l + ES, op_dt(o)));
    }
    T x = cadd(v0, v1);  // bit 0 summed in registers
#pragma unroll
    for (int i = 0; i < kStepOps; i++)
      if (i < n_step && !h0[i]) x = cmul(x, e0[i]);
    for (int k = max(k_extra, k_h0_end); k < kb + n_step; k++) {
      const DevOp &o = gops[k];
      const uint32_t ES = esize<T, CVT>(op_dt(o));
      const char *p = uniform_ptr(opnd(data, o, set) +
                                  ((uint64_t)pext_runs(Iu, o) + (uint32_t)stab[o.stab + s]) * ES);
      x = cmul(x, gload_dt<T, CVT>(p, s_lane[k * 64 + lane] * ES, op_dt(o)));
    }
    if (sl > 0) x = cmul(x, readlane2(U, s));
    for (int k = ks; k < ke; k++) {
      const DevOp &o = gops[k];
      const uint32_t ES = esize<T, CVT>(op_dt(o));
      const char *p = uniform_ptr(opnd(data, o, set) +
                                  ((uint64_t)pext_runs(Iu, o) + (uint32_t)stab[o.stab + s]) * ES);
      x = cmul(x, gload_dt<T, CVT>(p, s_lane[k * 64 + lane] * ES, op_dt(o)));
    }
    acc = cadd(acc, x);
  }
  // lane-summed bits: butterflies
  for (int b = 0; b < rls; b++) acc = cadd(acc, shfl_xor2(acc, 1 << b));
  if ((lane & ((1 << rls) - 1)) == 0) {
    const uint32_t o = (Iu | G.lane_kept((uint32_t)lane >> rls)) >> L;
    if (o < (1u << (G.w - L))) ((T *)outp(data, G, set))[o] = acc;
  }
}

// -------------------------------------------------------------------- cells

// Per-lane operand constants of the cell mapping: lane k holds operand k's
// (k < n_ops <= 64).
struct CellLane {
  uint64_t base;    // address of the operand in angle set 0
  uint64_t sstride; // bytes between angle sets
  uint32_t es, dt;  // element bytes in the group's arithmetic, storage type
  uint32_t cm;      // cell bits the operand's index holds
};

// Block-wide setup.  LDS: the byte offsets of every operand, cell and lane
// ([k][c][lane]: lane part plus cell part of the operand's index), then the
// unit-bit runs of every operand ([k][kCellURuns / 2]).  Registers: the
// lane's own operand constants.
template <class T, bool CVT, int NC>
__device__ __forceinline__ void cell_setup(const GI &G, const DevOp *__restrict__ gops,
                                           const int32_t *__restrict__ ctab, char *data,
                                           uint32_t *s_tab, CellLane &cl) {
  for (int e = threadIdx.x; e < G.n_ops * NC * 64; e += blockDim.x) {
    const int k = e / (NC * 64), c = (e / 64) % NC, lane = e & 63;
    const DevOp &o = gops[k];
    s_tab[e] = (pext_runs((uint32_t)lane, o) + (uint32_t)ctab[o.stab + c]) * esize<T, CVT>(op_dt(o));
  }
  uint32_t *s_ur = s_tab + G.n_ops * NC * 64;
  for (int e = threadIdx.x; e < G.n_ops * (kCellURuns / 2); e += blockDim.x) {
    const int k = e / (kCellURuns / 2), i = e % (kCellURuns / 2);
    s_ur[e] = (uint32_t)ctab[gops[k].stab + NC + i];
  }
  const int k = min((int)(threadIdx.x & 63), G.n_ops - 1);
  const DevOp &o = gops[k];
  cl.dt = (uint32_t)o.dt;
  cl.es = esize<T, CVT>(cl.dt);
  cl.base = (uint64_t)(data + o.off);
  cl.sstride = (uint64_t)o.sstride;
  cl.cm = (uint32_t)ctab[o.stab + NC + kCellURuns / 2];
}

// One reduce-scatter step over lane bit t: of the 2 * HALF accumulators the
// lane keeps the half selected by its bit t, adding the partner lane's copy.
template <class T, int HALF>
__device__ __forceinline__ void reduce_scatter_step(T *acc, int lane, int t) {
  const bool hi = ((lane >> t) & 1) != 0;
#pragma unroll
  for (int i = 0; i < HALF; i++) {
    const T keep = hi ? acc[i + HALF] : acc[i];
    const T send = hi ? acc[i] : acc[i + HALF];
    acc[i] = cadd(keep, shfl_xor2(send, 1 << t));
  }
}

// Sums the lane-summed bits 0..ls-1 of the 2^RB register accumulators and
// writes the results: a reduce-scatter over the first q = min(RB, ls) bits
// (afterwards lane bit t selects half of the cells), butterflies for the rest.
template <class T, int RB>
__device__ __forceinline__ void cell_finish(const GI &G, T *acc, const uint8_t *__restrict__ ubit,
                                            uint32_t Iu, int ls, int lane, T *out) {
  constexpr int NR = 1 << RB;
  const int L = G.L, q = min(RB, ls);
  if (RB >= 1 && ls > 0) reduce_scatter_step<T, (NR >> 1)>(acc, lane, 0);
  if (RB >= 2 && ls > 1) reduce_scatter_step<T, (NR >> 2)>(acc, lane, 1);
  if (RB >= 3 && ls > 2) reduce_scatter_step<T, (NR >> 3)>(acc, lane, 2);
  if (RB >= 4 && ls > 3) reduce_scatter_step<T, (NR >> 4)>(acc, lane, 3);
  const int nacc = NR >> q;
  for (int t = q; t < ls; t++) {
#pragma unroll
    for (int i = 0; i < NR; i++)
      if (i < nacc) acc[i] = cadd(acc[i], shfl_xor2(acc[i], 1 << t));
  }
  // lanes whose summed bits q..ls-1 are zero hold the results; acc[i] is
  // register cell i + sum_t (lane bit t) * (NR >> (t + 1))
  if ((((uint32_t)lane >> q) & ((1u << (ls - q)) - 1u)) == 0) {
    const uint32_t Ik = Iu | ((uint32_t)lane & ~((1u << ls) - 1u));
    uint32_t jb = 0;
    for (int t = 0; t < q; t++) jb += (((uint32_t)lane >> t) & 1u) * (uint32_t)(NR >> (t + 1));
    const uint32_t nout = 1u << (G.w - L);
#pragma unroll
    for (int i = 0; i < NR; i++) {
      if (i < nacc) {
        const uint32_t j = jb + (uint32_t)i;
        uint32_t I = Ik;
#pragma unroll
        for (int b = 0; b < RB; b++) I |= ((j >> b) & 1u) << ubit_at(ubit, b);
        const uint32_t o = I >> L;
        if (o < nout) out[o] = acc[i];
      }
    }
  }
}

// acc[c] (c < N; first: set to) times operand k, whose index holds the cell
// bits CM: only the distinct cells (c & ~CM == 0) are loaded, each value
// serving every cell that differs from it in bits outside CM.
template <class T, bool CVT, int NC, int N, int CM>
__device__ __forceinline__ void cell_op_cm(T *acc, bool first, const char *p, int dt,
                                           const uint32_t *lt) {
  T v[N];
#pragma unroll
  for (int c = 0; c < N; c++)
    if ((c & ~CM) == 0) v[c] = gload_dt<T, CVT>(p, lt[c * 64], dt);
  if (first) {
#pragma unroll
    for (int c = 0; c < N; c++) acc[c] = v[c & CM];
  } else {
#pragma unroll
    for (int c = 0; c < N; c++) acc[c] = cmul(acc[c], v[c & CM]);
  }
}

// acc[c] (c < N) times operand k (uniform): scalar base from lane k's
// address, per-lane offsets of each cell from the LDS table.
template <class T, bool CVT, int NC, int N>
__device__ __forceinline__ void cell_op(T *acc, bool first, int k, const CellLane &cl,
                                        uint64_t addr, const uint32_t *s_tab, int lane) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)addr, k);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(addr >> 32), k);
  const char *p = (const char *)(((uint64_t)hi << 32) | lo);
  const int dt = CVT ? (int)__builtin_amdgcn_readlane(cl.dt, k) : 0;
  const uint32_t cm = __builtin_amdgcn_readlane(cl.cm, k) & (uint32_t)(N - 1);
  const uint32_t *lt = s_tab + k * NC * 64 + lane;
#define QTN_CM(m) \
  case m: cell_op_cm<T, CVT, NC, N, (m) & (N - 1)>(acc, first, p, dt, lt); break;
  switch (cm) {
    QTN_CM(0) QTN_CM(1) QTN_CM(2) QTN_CM(3) QTN_CM(4) QTN_CM(5) QTN_CM(6) QTN_CM(7)
    QTN_CM(8) QTN_CM(9) QTN_CM(10) QTN_CM(11) QTN_CM(12) QTN_CM(13) QTN_CM(14)
    default: cell_op_cm<T, CVT, NC, N, (15 & (N - 1))>(acc, first, p, dt, lt); break;
  }
#undef QTN_CM
}

// One wave unit of the cell mapping.  The lanes take union bits 0..5, the
// lowest index bits of the large operands, so one load of an operand by the
// wave covers whole cache lines.  Each lane holds NC = 2^CB cells: the high
// SL cell bits are the summed bits 6..L-1 (serial; bit 6 the highest cell
// bit), the low RB = CB - SL cell bits kept bits.  Every point multiplies all
// operands, as bucket elimination orders them: the operands holding bit 6
// in every cell, then bit 6 is summed, the operands holding bit 7 (but not
// 6) in the cells left, bit 7 is summed, and the other operands multiply the
// 2^RB register cells.  The lane-summed bits are reduced last.  Operand
// addresses for the unit are formed by lane k for operand k.
template <class T, bool CVT, int CB, int SL>
__device__ __forceinline__ void cell_unit(const GI &G, const CellLane &cl,
                                          const uint8_t *__restrict__ ubit, char *__restrict__ data,
                                          const uint32_t *s_tab, const T *P, uint32_t u, int lane,
                                          uint32_t set) {
  constexpr int NC = 1 << CB, RB = CB - SL, NR = 1 << RB;
  const int n_step = G.n_step, n_ops = G.n_ops, nfix = G.n_step0;
  // lane k: unit part of operand k's index, then its address for this unit
  const uint32_t *s_ur = s_tab + n_ops * NC * 64 + min(lane, n_ops - 1) * (kCellURuns / 2);
  uint32_t ub = 0;
  for (int i = 0; i < G.n_unit; i += 2) {
    const uint32_t w = s_ur[i >> 1];
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const uint32_t rr = (w >> (16 * h)) & 0xFFFFu;  // an unused run is 0
      const uint32_t src = rr & 31u, len = (rr >> 5) & 63u, dst = rr >> 11;
      ub |= ((u >> src) & (uint32_t)((1ull << len) - 1ull)) << dst;
    }
  }
  const uint64_t addr = cl.base + (uint64_t)set * cl.sstride + (uint64_t)ub * cl.es;
  T acc[NC];
  // operands holding bit 6 (every operand when no bit is serial) in all
  // cells; without serial bits, the first nfix (lane bits only) are the
  // product P[0] applied last
  int k = SL == 0 ? nfix : 0;
  for (const int k0 = k; k < n_step; k++) cell_op<T, CVT, NC, NC>(acc, k == k0, k, cl, addr, s_tab, lane);
  if (SL == 0 && nfix > 0) {
    if (nfix == n_step) {
#pragma unroll
      for (int c = 0; c < NC; c++) acc[c] = P[0];
    } else {
#pragma unroll
      for (int c = 0; c < NC; c++) acc[c] = cmul(acc[c], P[0]);
    }
  }
  if (SL >= 1) {
    // sum bit 6 (the highest cell bit)
#pragma unroll
    for (int c = 0; c < NC / 2; c++) acc[c] = cadd(acc[c], acc[c + NC / 2]);
  }
  if (SL == 2) {
    // operands holding bit 7 but not 6, then sum bit 7
    const int k1 = n_step + G.n_serial;
    for (k = n_step; k < k1; k++)
      cell_op<T, CVT, NC, (SL == 2 ? NC / 2 : 1)>(acc, false, k, cl, addr, s_tab, lane);
#pragma unroll
    for (int c = 0; c < NC / 4; c++) acc[c] = cadd(acc[c], acc[c + NC / 4]);
  }
  if (SL >= 1) {
    // the operands without serial bits in the register cells: first the
    // unit-invariant product, then the others
    k = n_step + (SL == 2 ? G.n_serial : 0);
    if (SL >= 1 && nfix > 0) {
#pragma unroll
      for (int c = 0; c < NR; c++) acc[c] = cmul(acc[c], P[c]);
      k += nfix;
    }
    for (; k < n_ops; k++) cell_op<T, CVT, NC, NR>(acc, false, k, cl, addr, s_tab, lane);
  }
  const uint32_t Iu = unit_bits(u, ubit, G.n_ubits, RB);
  cell_finish<T, RB>(G, acc, ubit, Iu, SL > 0 ? 6 : min(G.L, 6), lane, (T *)outp(data, G, set));
}

// Setup and units [u0, u1) (one per wave, strided) of a cell-mapped group.
// With serial bits, the product P of the operands without them that hold no
// unit bit (the first n_step0 of the last level) depends only on the lane, the
// register cell and the angle set; without serial bits, P[0] is the product
// of the first n_step0 operands, which hold lane bits only.  A wave forms P
// when its set changes.
template <class T, bool CVT, int CB, int SL>
__device__ __forceinline__ void cell_units(const GI &G, const DevOp *__restrict__ gops,
                                           const int32_t *__restrict__ ctab,
                                           const uint8_t *__restrict__ ubit, char *__restrict__ data,
                                           uint32_t *s_tab, uint32_t u0, uint32_t u1,
                                           uint32_t stride, uint32_t set_units, int lane) {
  constexpr int NC = 1 << CB, NR = 1 << (CB - SL);
  CellLane cl;
  cell_setup<T, CVT, NC>(G, gops, ctab, data, s_tab, cl);
  __syncthreads();
  const int nfix = G.n_step0;
  const int kf = SL == 0 ? 0 : G.n_step + (SL == 2 ? G.n_serial : 0);
  T P[SL > 0 ? NR : 1];
  uint32_t pset = 0xFFFFFFFFu;
  // flat unit f: angle set f / set_units, unit f % set_units
  for (uint32_t f = u0; f < u1; f += stride) {
    const uint32_t set = f / set_units;
    if (nfix > 0 && set != pset) {
      const uint64_t a0 = cl.base + (uint64_t)set * cl.sstride;  // no unit part
      for (int k = kf; k < kf + nfix; k++)
        cell_op<T, CVT, NC, (SL > 0 ? NR : 1)>(P, k == kf, k, cl, a0, s_tab, lane);
      pset = set;
    }
    cell_unit<T, CVT, CB, SL>(G, cl, ubit, data, s_tab, P, f - set * set_units, lane, set);
  }
}

// ------------------------------------------------------------ matrix form

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Matrix cores, one 16 x 16 x 4 real product (A 16 x 4, B 4 x 16, one value
// per lane: A[i][k] from lane i + 16k, B[k][j] from lane j + 16k), FP64 for
// complex128 and FP32 for complex64 groups.  Output element r of lane l is
// C[row][l % 16] with row (l / 16) + 4r (FP64) or 4 (l / 16) + r (FP32).
__device__ __forceinline__ f64x4 mm_step(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mm_step(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <class T> struct MmTypes;
template <> struct MmTypes<double2> {
  typedef double R;
  typedef f64x4 V;
  __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct MmTypes<float2> {
  typedef float R;
  typedef f32x4 V;
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// LDS bytes of a matrix-form tile in arithmetic type T with NCB 16-column
// blocks: the operands' tile bases (kMmMaxOps words, padded to 256 bytes),
// the A chunk [kMmTM][kMmKC + 1] and the B chunk [kMmKC][16 NCB + 1].
template <class T, int NCB> constexpr int mm_lds_bytes() {
  return 256 + (kMmTM * (kMmKC + 1) + kMmKC * (16 * NCB + 1)) * (int)sizeof(T);
}
static_assert(kMmMaxOps * 4 <= 256, "matrix-form operand bases");
static_assert(mm_lds_bytes<float2, 4>() <= kStreamMaxOps * 64 * 4,
              "complex64 matrix tiles must fit the workgroup kernels' LDS");

// One kMmTM x 16 NCB output tile of a matrix-form group, with the whole
// workgroup:
//   out[bt, m, n] = sum_k At[bt, m, k] Bt[bt, k, n],
// At (Bt) the product of the group's side-A (side-B) operands, k over the L
// summed union bits.  Per chunk of KC = min(max(2^L, 4), kMmKC) summed
// indices both factors are gathered into LDS: thread t takes k = t % KC (the
// lowest union bits, so that threads with neighbouring k read neighbouring
// elements) and the rows (columns) t / KC + (256 / KC) j.  An operand's
// element offset is its tile base plus table entries for the row (column)
// and for k; both tables are pext images of disjoint bit sets, so an entry
// splits into a per-thread part (row and k below the pass and chunk sizes)
// and parts uniform over the block (the pass and the chunk).  Then wave v
// multiplies its 16 rows into NCB 16 x 16 column blocks: three real products
// per complex product (3M), accumulated in the group's precision.  Operands:
// [side A..., side B...]; G.gtab holds the union bits of the tile's rows
// (kMmTM words) and columns (kMmTN words, the first 16 NCB used); operand
// k's table (at its stab) holds kMmTM row (side A) or kMmTN column (side B)
// offsets, then 2^L summed-index offsets.  Unit bits (uperm): m bits, then n
// bits, then batch bits.
template <class T, bool CVT, int NCB>
__device__ void mm_tile(const GI &G, const DevOp *__restrict__ gops, const int32_t *__restrict__ stab,
                        const uint8_t *__restrict__ bits, char *__restrict__ data, char *lds,
                        uint32_t tile, uint32_t set) {
  typedef typename MmTypes<T>::R R;
  typedef typename MmTypes<T>::V V;
  constexpr int TN = 16 * NCB, TNB = NCB == 1 ? 4 : (NCB == 2 ? 5 : 6);
  constexpr int AP = kMmTM * kMmKC / 256;  // most side-A passes (KC = kMmKC)
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nM = G.n_mb, nN = G.n_nb, nB = G.n_bb, L = G.L;
  const uint32_t M = 1u << nM, N = 1u << nN, K = 1u << L;
  const uint32_t mt = (M + kMmTM - 1) / kMmTM, nt = (N + TN - 1) / TN;
  const uint32_t bt = tile / (mt * nt), rem = tile % (mt * nt);
  const uint32_t mi = rem / nt, ni = rem % nt;
  const uint32_t m0 = mi * kMmTM, n0 = ni * TN;
  // union bits of the tile: batch bits, and the m (n) bits above the
  // in-tile ones (a tile spans the lowest 6 m bits and TNB n bits)
  const int mlo = nM < 6 ? nM : 6, nlo = nN < TNB ? nN : TNB;
  const uint32_t Ib = unit_bits(bt, bits, nB, nM + nN) | unit_bits(mi, bits, nM - mlo, mlo) |
                      unit_bits(ni, bits, nN - nlo, nM + nlo);
  const int na = G.n_unit, nb = G.n_step;
  const int32_t *mu = stab + G.gtab, *nu = mu + kMmTM;
  uint32_t *base = (uint32_t *)lds;  // each operand's element offset at the tile's union bits
  T *sA = (T *)(lds + 256), *sB = sA + kMmTM * (kMmKC + 1);
  if (tid < na + nb) base[tid] = pext_runs(Ib, gops[tid]);
  __syncthreads();
  // 3M: t1 = sum Ar Br, t2 = sum Ai Bi, t3 = sum (Ar + Ai)(Br + Bi); then
  // Re = t1 - t2, Im = t3 - t1 - t2
  V t1[NCB], t2[NCB], t3[NCB];
#pragma unroll
  for (int s = 0; s < NCB; s++)
#pragma unroll
    for (int r = 0; r < 4; r++) t1[s][r] = t2[s][r] = t3[s][r] = (R)0;
  // chunk size KC = 2^kb, passes of RP = 256 / KC rows (columns)
  const int kb = L < 2 ? 2 : (L > 4 ? 4 : L), KC = 1 << kb, RP = 256 >> kb;
  const int kl = tid & (KC - 1), rl = tid >> kb;
  const int pa = kMmTM / RP, pb = (TN + RP - 1) / RP;
  const int klt = (uint32_t)kl < K ? kl : 0;  // table index of kl (2^L < KC: padding)
  for (uint32_t k0 = 0; k0 < K; k0 += (uint32_t)KC) {
    const uint32_t k = k0 + (uint32_t)kl;
    // side A: rows rl + RP j
    T va[AP];
    bool oka[AP];
#pragma unroll
    for (int j = 0; j < AP; j++) {
      oka[j] = j < pa && m0 + (uint32_t)(rl + RP * j) < M && k < K;
      va[j] = make_c<T>(1.0, 0.0);
    }
    for (int q = 0; q < na; q++) {
      const DevOp &o = gops[q];
      const int32_t *t = stab + o.stab;
      const char *p = opnd(data, o, set);
      const int dt = op_dt(o);
      const uint32_t e0 = base[q] + (uint32_t)t[rl] + (uint32_t)t[kMmTM + klt] +
                          (uint32_t)t[kMmTM + k0];
#pragma unroll
      for (int j = 0; j < AP; j++)
        if (oka[j]) va[j] = cmul(va[j], ld_elem<T, CVT>(p, e0 + (uint32_t)t[RP * j], dt));
    }
#pragma unroll
    for (int j = 0; j < AP; j++)
      if (j < pa) sA[(rl + RP * j) * (kMmKC + 1) + kl] = oka[j] ? va[j] : make_c<T>(0.0, 0.0);
    // side B: columns rl + RP j
    T vb[NCB];
    bool okb[NCB];
#pragma unroll
    for (int j = 0; j < NCB; j++) {
      const int col = rl + RP * j;
      okb[j] = j < pb && col < TN && n0 + (uint32_t)col < N && k < K;
      vb[j] = make_c<T>(1.0, 0.0);
    }
    for (int q = na; q < na + nb; q++) {
      const DevOp &o = gops[q];
      const int32_t *t = stab + o.stab;
      const char *p = opnd(data, o, set);
      const int dt = op_dt(o);
      const int c0 = rl < TN ? rl : 0;
      const uint32_t e0 = base[q] + (uint32_t)t[c0] + (uint32_t)t[kMmTN + klt] +
                          (uint32_t)t[kMmTN + k0];
#pragma unroll
      for (int j = 0; j < NCB; j++)
        if (okb[j]) vb[j] = cmul(vb[j], ld_elem<T, CVT>(p, e0 + (uint32_t)t[RP * j], dt));
    }
#pragma unroll
    for (int j = 0; j < NCB; j++) {
      const int col = rl + RP * j;
      if (j < pb && col < TN) sB[kl * (TN + 1) + col] = okb[j] ? vb[j] : make_c<T>(0.0, 0.0);
    }
    __syncthreads();
    for (int kk = 0; kk < KC; kk += 4) {
      const T a = sA[(wave * 16 + (lane & 15)) * (kMmKC + 1) + kk + (lane >> 4)];
      const R ar = (R)a.x, ai = (R)a.y, as = ar + ai;
#pragma unroll
      for (int s = 0; s < NCB; s++) {
        const T b = sB[(kk + (lane >> 4)) * (TN + 1) + 16 * s + (lane & 15)];
        const R br = (R)b.x, bi = (R)b.y;
        t1[s] = mm_step(ar, br, t1[s]);
        t2[s] = mm_step(ai, bi, t2[s]);
        t3[s] = mm_step(as, br + bi, t3[s]);
      }
    }
    __syncthreads();
  }
  T *out = (T *)outp(data, G, set);
  const uint32_t nout = 1u << (G.w - L);
#pragma unroll
  for (int s = 0; s < NCB; s++) {
    const int col = 16 * s + (lane & 15);
    const bool okc = n0 + (uint32_t)col < N;
#pragma unroll
    for (int r = 0; r < 4; r++) {
      // combined in every lane, stored where the row and column exist
      T v;
      v.x = t1[s][r] - t2[s][r];
      v.y = t3[s][r] - t1[s][r] - t2[s][r];
      const int row = wave * 16 + MmTypes<T>::row(lane, r);
      if (okc && m0 + (uint32_t)row < M) {
        const uint32_t o = (Ib | (uint32_t)mu[row] | (uint32_t)nu[col]) >> L;
        if (o < nout) out[o] = v;
      }
    }
    // one column block at a time: keeps the accumulators that are read out
    // into vector registers to one block's worth
    __builtin_amdgcn_sched_barrier(0);
  }
}

// One group's wave units [u0, u1) of angle set `set` over the block's waves,
// in the group's own precision.
__device__ __forceinline__ void run_group(const GI &G, int g, const DevOp *__restrict__ ops,
                                          const int32_t *__restrict__ stab,
                                          const uint8_t *__restrict__ uperm, char *__restrict__ data,
                                          uint32_t *s_lane, uint32_t u0, uint32_t u1,
                                          uint32_t set) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const DevOp *gops = ops + G.op_begin;
  const uint8_t *ub = uperm + 32 * g;
#define QTN_UNITS(F, ...)                                                          \
  do {                                                                             \
    if (G.prec == 0 && !G.cvt)                                                     \
      for (uint32_t u = u0 + wave; u < u1; u += nw) F<double2, false>(__VA_ARGS__); \
    else if (G.prec == 0)                                                          \
      for (uint32_t u = u0 + wave; u < u1; u += nw) F<double2, true>(__VA_ARGS__);  \
    else if (!G.cvt)                                                               \
      for (uint32_t u = u0 + wave; u < u1; u += nw) F<float2, false>(__VA_ARGS__);  \
    else                                                                           \
      for (uint32_t u = u0 + wave; u < u1; u += nw) F<float2, true>(__VA_ARGS__);   \
  } while (0)
  if (G.variant == kVarMfma) {
    // matrix form (complex64 inside workgroups): a unit is one 64 x 16
    // output tile, computed by the whole block (one column block per wave
    // keeps the accumulators, and so these kernels' registers, few)
    if (G.cvt)
      for (uint32_t u = u0; u < u1; u++)
        mm_tile<float2, true, 1>(G, gops, stab, ub, data, (char *)s_lane, u, set);
    else
      for (uint32_t u = u0; u < u1; u++)
        mm_tile<float2, false, 1>(G, gops, stab, ub, data, (char *)s_lane, u, set);
  } else if (G.variant == kVarStream) {
    stream_setup(G, gops, s_lane);
    __syncthreads();
    QTN_UNITS(stream_unit, G, gops, stab, ub, data, s_lane, u, lane, set);
  } else {
    QTN_UNITS(generic_unit, G, gops, ub, data, u, lane, set);
  }
#undef QTN_UNITS
  __syncthreads();
}

// ------------------------------------------------------------------ kernels

// Compiled for 5 waves per SIMD (a few registers spill on the rarely taken
// mappings): the small groups are latency-bound, and the extra waves measured
// 3% faster than the 4 the register count would give.
__global__ __launch_bounds__(kBlock, 5) void k_block_groups(char *__restrict__ data,
                                                         const DevGroup *__restrict__ groups,
                                                         const DevOp *__restrict__ ops,
                                                         const int32_t *__restrict__ stab,
                                                         const uint8_t *__restrict__ uperm,
                                                         const int2 *__restrict__ ranges,
                                                         int range_base, int n_ranges) {
  __shared__ __align__(16) uint32_t s_lane[kStreamMaxOps * 64];
  // block b runs range b % n_ranges for angle set b / n_ranges
  const uint32_t set = blockIdx.x / (uint32_t)n_ranges;
  const int2 rg = ranges[range_base + (int)(blockIdx.x % (uint32_t)n_ranges)];
  for (int g = rg.x; g < rg.y; g++) {
    const GI G = load_group(groups + g);
    run_group(G, g, ops, stab, uperm, data, s_lane, 0u, G.n_units, set);
  }
}

// Units of a wide launch.  Blocks are dealt round-robin to the 8 XCDs; each
// XCD takes one contiguous slice of the flat unit space (its own L2), and the
// XCD's blocks walk that slice together, one unit per wave and chunk by chunk,
// so that at any time they work on neighbouring units, which share the data
// of the operands lacking the low unit bits.  (Each block walking a slice of
// its own instead spreads the resident blocks over as many distant regions,
// whose reused data does not fit in the L2 at once.)  The host keeps
// n_units + the grid's wave count below 2^32.
struct UnitWalk {
  uint32_t first, end, stride;
};
__device__ __forceinline__ UnitWalk wide_walk(uint32_t n_units, uint32_t nw, uint32_t w) {
  const uint32_t nb = gridDim.x, b = blockIdx.x;
  const bool xcd = nb % 8u == 0u;
  const uint32_t nx = xcd ? 8u : 1u, x = xcd ? b % 8u : 0u, j = xcd ? b / 8u : b;
  const uint32_t per = (n_units + nx - 1) / nx;
  UnitWalk W;
  W.end = min(n_units, x * per + per);
  W.first = x * per + j * nw + w;
  W.stride = (nb / nx) * nw;
  return W;
}

template <class T, bool CVT>
__global__ __launch_bounds__(kBlock) void k_wide_stream(char *__restrict__ data,
                                                        const DevGroup *__restrict__ groups,
                                                        const DevOp *__restrict__ ops,
                                                        const int32_t *__restrict__ stab,
                                                        const uint8_t *__restrict__ uperm, int gid,
                                                        uint32_t n_sets) {
  // lane tables of the group's operands: n_ops * 64 words, sized at launch
  extern __shared__ __align__(16) uint32_t s_lane[];
  const GI G = load_group(groups + gid);
  const DevOp *gops = ops + G.op_begin;
  const int lane = threadIdx.x & 63;
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t w0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const UnitWalk W = wide_walk(G.n_units * n_sets, nw, w0);
  stream_setup(G, gops, s_lane);
  __syncthreads();
  // flat unit f: angle set f / n_units, unit f % n_units
  for (uint32_t f = W.first; f < W.end; f += W.stride) {
    const uint32_t set = f / G.n_units;
    stream_unit<T, CVT>(G, gops, stab, uperm + 32 * gid, data, s_lane, f - set * G.n_units, lane,
                        set);
  }
}

// With 3 cell bits and 2 serial bits the kernel fits 5 waves per SIMD without
// spilling when asked to (92 registers; 4 waves otherwise): 7% faster on the
// 8-summed-bit groups.  The other forms would spill, for no measured gain.
template <class T, bool CVT, int CB, int SL>
__global__ __launch_bounds__(kBlock, (CB == 3 && SL == 2 ? 5 : 1)) void k_wide_cells(char *__restrict__ data,
                                                       const DevGroup *__restrict__ groups,
                                                       const DevOp *__restrict__ ops,
                                                       const int32_t *__restrict__ ctab,
                                                       const uint8_t *__restrict__ uperm, int gid,
                                                       uint32_t n_sets) {
  // offset tables of the group's operands, sized at launch
  extern __shared__ __align__(16) uint32_t s_tab[];
  const GI G = load_group(groups + gid);
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t w0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const UnitWalk W = wide_walk(G.n_units * n_sets, nw, w0);
  cell_units<T, CVT, CB, SL>(G, ops + G.op_begin, ctab, uperm + 32 * gid, data, s_tab, W.first,
                             W.end, W.stride, G.n_units, threadIdx.x & 63);
}

template <class T, bool CVT>
__global__ __launch_bounds__(kBlock) void k_wide_generic(char *__restrict__ data,
                                                         const DevGroup *__restrict__ groups,
                                                         const DevOp *__restrict__ ops,
                                                         const int32_t *__restrict__ stab,
                                                         const uint8_t *__restrict__ uperm,
                                                         int gid, uint32_t n_sets) {
  const GI G = load_group(groups + gid);
  const DevOp *gops = ops + G.op_begin;
  const int lane = threadIdx.x & 63;
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t w0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const UnitWalk W = wide_walk(G.n_units * n_sets, nw, w0);
  for (uint32_t f = W.first; f < W.end; f += W.stride) {
    const uint32_t set = f / G.n_units;
    generic_unit<T, CVT>(G, gops, uperm + 32 * gid, data, f - set * G.n_units, lane, set);
  }
}

// Waves per SIMD the matrix-form kernel is compiled for: three accumulator
// sets of NCB blocks (3M) fill many registers, and left alone the compiler
// spends more on staging than this occupancy allows.
template <class T, int NCB> constexpr int mm_waves() {
  return sizeof(T) == 8 ? (NCB == 4 ? 4 : 5) : (NCB == 4 ? 3 : 4);
}

template <class T, bool CVT, int NCB>
__global__ __launch_bounds__(kBlock, (mm_waves<T, NCB>())) void k_wide_mfma(char *__restrict__ data,
                                                      const DevGroup *__restrict__ groups,
                                                      const DevOp *__restrict__ ops,
                                                      const int32_t *__restrict__ stab,
                                                      const uint8_t *__restrict__ uperm, int gid,
                                                      uint32_t n_sets) {
  __shared__ __align__(16) char s_tile[mm_lds_bytes<T, NCB>()];
  const GI G = load_group(groups + gid);
  const UnitWalk W = wide_walk(G.n_units * n_sets, 1, 0);
  for (uint32_t f = W.first; f < W.end; f += W.stride) {
    const uint32_t set = f / G.n_units;
    mm_tile<T, CVT, NCB>(G, ops + G.op_begin, stab, uperm + 32 * gid, data, s_tile,
                         f - set * G.n_units, set);
  }
}

// ----------------------------------------------------- persistent executor

// Runs one work item with the whole block: a segment of small groups
// [it.x, it.y) in order, or units [it.z, it.w) of wide group it.x (it.y < 0).
__device__ __forceinline__ void run_item(int4 it, char *__restrict__ data,
                                         const DevGroup *__restrict__ groups,
                                         const DevOp *__restrict__ ops,
                                         const int32_t *__restrict__ stab,
                                         const uint8_t *__restrict__ uperm, uint32_t *s_lane) {
  const bool chunk = it.y < 0;
  const int g_end = chunk ? it.x + 1 : it.y;
  for (int g = it.x; g < g_end; g++) {
    const GI G = load_group(groups + g);
    const uint32_t u0 = chunk ? (uint32_t)it.z : 0u;
    const uint32_t u1 = chunk ? min((uint32_t)it.w, G.n_units) : G.n_units;
    run_group(G, g, ops, stab, uperm, data, s_lane, u0, u1, 0u);
  }
}

// Grid-wide barrier over resident blocks.  Block writes are released at agent
// scope before arriving and acquired after leaving.  The wait is bounded: past
// `spin_limit` polls the block records an error and the kernel stops early.
__device__ __forceinline__ bool grid_barrier(uint32_t *ctl, uint32_t spin_limit) {
  uint32_t *count = ctl, *gen = ctl + 1, *err = ctl + 2;
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    s_ok = 1;
    __threadfence();
    const uint32_t g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t arrived =
        __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == gridDim.x - 1) {
      __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint32_t polls = 0;
      while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
        __builtin_amdgcn_s_sleep(4);
        if (++polls > spin_limit ||
            __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
          __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          s_ok = 0;
          break;
        }
      }
    }
    __threadfence();
  }
  __syncthreads();
  return s_ok != 0;
}

// Every light cone's tasks in lockstep: step s runs the s-th task of every
// cone (a segment of small groups, or a chunk of a wide group), blocks taking
// items with an atomic counter; a grid barrier separates steps.  ctl:
// [barrier count, barrier generation, error flag, pad, per-step counters...],
// cleared by k_reset before the launch.
// Compiled for 5 waves per SIMD (the launch takes as many blocks as fit; a
// few registers spill on the rarely taken mappings): the batch of 64 graphs
// measured 1309 energies per second, against 1197 with the 4 waves the
// register count alone gives.
__global__ __launch_bounds__(kBlock, 5) void k_persistent(char *__restrict__ data,
                                                       const DevGroup *__restrict__ groups,
                                                       const DevOp *__restrict__ ops,
                                                       const int32_t *__restrict__ stab,
                                                       const uint8_t *__restrict__ uperm,
                                                       const int4 *__restrict__ items,
                                                       const int *__restrict__ step_begin,
                                                       int n_steps, uint32_t *ctl,
                                                       uint32_t spin_limit) {
  __shared__ __align__(16) uint32_t s_lane[kStreamMaxOps * 64];
  __shared__ int s_item;
  uint32_t *step_ctr = ctl + 4;
  for (int st = 0; st < n_steps; st++) {
    const int b = step_begin[st], e = step_begin[st + 1];
    for (;;) {
      if (threadIdx.x == 0)
        s_item = b + (int)__hip_atomic_fetch_add(step_ctr + st, 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      const int i = s_item;
      __syncthreads();
      if (i >= e) break;
      run_item(items[i], data, groups, ops, stab, uperm, s_lane);
    }
    if (st + 1 < n_steps && !grid_barrier(ctl, spin_limit)) return;
  }
}

// Dataflow form of the executor, with a ready queue.  Work items (a cone's
// segment of small groups, or a chunk of a wide group) belong to tasks; a
// cone's tasks form a chain.  queue[] receives item indices (+1; 0 = empty)
// as their tasks become ready: the first task of every cone before the
// launch, a task's successor when the last item of the task completes.
// Blocks claim queue slots in order from ctl[0] and run the item once its
// slot is filled.  A block only waits when no ready item is left, and the
// block that completes a task publishes its successor before claiming again,
// so the earliest unfilled slot is always being worked towards.
//
// ctl: [claim counter, fill counter, error flag, pad, done counter per task].
// Results are released (agent scope) before a done count, acquired by the
// completing block before it publishes the successor, and acquired again by
// the block that takes a published item.
//
// The bookkeeping runs in one branch at the top of the loop that is uniform
// per wave (wave 0; lane 0 alone issues the counter atomics): a lane-divergent
// region at the end of the loop body could be rotated across the back edge,
// so that the other lanes of wave 0 met the next barrier before lane 0 had
// taken the next item.
__global__ __launch_bounds__(kBlock) void k_dataflow(char *__restrict__ data,
                                                     const DevGroup *__restrict__ groups,
                                                     const DevOp *__restrict__ ops,
                                                     const int32_t *__restrict__ stab,
                                                     const uint8_t *__restrict__ uperm,
                                                     const int4 *__restrict__ items, int n_items,
                                                     const int *__restrict__ item_task,
                                                     const int *__restrict__ task_next,
                                                     const int *__restrict__ task_first,
                                                     const int *__restrict__ task_need,
                                                     uint32_t *queue, uint32_t *ctl,
                                                     uint32_t spin_limit) {
  __shared__ __align__(16) uint32_t s_lane[kStreamMaxOps * 64];
  __shared__ int s_item, s_ok;
  uint32_t *claim = ctl, *fill = ctl + 1, *err = ctl + 2, *done = ctl + 4;
  const int lane = threadIdx.x & 63;
  int prev = -1;  // item this block finished last (block-uniform)
  for (;;) {
    if (threadIdx.x < 64) {
      if (prev >= 0) {
        // release this block's results, then count the item done
        __threadfence();
        const int t = item_task[prev];
        uint32_t old = 0;
        if (lane == 0)
          old = __hip_atomic_fetch_add(done + t, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        old = __builtin_amdgcn_readfirstlane(old);
        const int nt = task_next[t];
        if (old + 1u == (uint32_t)task_need[t] && nt >= 0) {
          // the task is complete: acquire every item's results, then publish
          // the successor's items
          __threadfence();
          const uint32_t cnt = (uint32_t)task_need[nt], first = (uint32_t)task_first[nt];
          uint32_t base = 0;
          if (lane == 0)
            base = __hip_atomic_fetch_add(fill, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          base = __builtin_amdgcn_readfirstlane(base);
          for (uint32_t k = lane; k < cnt; k += 64)
            __hip_atomic_store(queue + base + k, first + k + 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      uint32_t h = 0;
      if (lane == 0)
        h = __hip_atomic_fetch_add(claim, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      h = __builtin_amdgcn_readfirstlane(h);
      int i = n_items, ok = 1;
      if (h < (uint32_t)n_items) {
        uint32_t polls = 0;
        for (;;) {
          const uint32_t v = __builtin_amdgcn_readfirstlane(
              __hip_atomic_load(queue + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
          if (v != 0u) {
            i = (int)v - 1;
            break;
          }
          __builtin_amdgcn_s_sleep(8);
          const uint32_t e = __builtin_amdgcn_readfirstlane(
              __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
          if (++polls > spin_limit || e != 0u) {
            if (lane == 0) __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
            break;
          }
        }
        __threadfence();  // acquire the item's inputs
      }
      if (lane == 0) {
        s_item = i;
        s_ok = ok;
      }
    }
    __syncthreads();
    const int i = s_item, ok = s_ok;
    __syncthreads();
    if (i >= n_items || i < 0 || !ok) break;
    run_item(items[i], data, groups, ops, stab, uperm, s_lane);  // ends with a barrier
    prev = i;
  }
}

// Control words to zero; the queue holds the first n_init items (0..n_init-1,
// the first task of every cone) and is empty after them; the fill counter
// starts at n_init.
__global__ void k_queue_reset(uint32_t *ctl, int n_ctl, uint32_t *queue, int n_items,
                              int n_init) {
  const int stride = gridDim.x * blockDim.x;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n_ctl; k += stride)
    ctl[k] = k == 1 ? (uint32_t)n_init : 0u;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n_items; k += stride)
    queue[k] = k < n_init ? (uint32_t)k + 1u : 0u;
}

__global__ void k_reset(uint32_t *ctl, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    ctl[i] = 0u;
}

// Gate values (Eq. 1-2): P = exp(-i gamma [a != b]), R = exp(-i beta X).
template <class T>
__device__ void put2x2(T *t, double2 m00, double2 m01, double2 m10, double2 m11) {
  // row-major over the gate's axes, then the same with the other axis as bit 0
  t[0] = make_c<T>(m00.x, m00.y);
  t[1] = make_c<T>(m01.x, m01.y);
  t[2] = make_c<T>(m10.x, m10.y);
  t[3] = make_c<T>(m11.x, m11.y);
  t[4] = make_c<T>(m00.x, m00.y);
  t[5] = make_c<T>(m10.x, m10.y);
  t[6] = make_c<T>(m01.x, m01.y);
  t[7] = make_c<T>(m11.x, m11.y);
}

template <class T>
__device__ void fill_table(T *table, const double *gamma, const double *beta, int p) {
  for (int l = threadIdx.x; l < p; l += blockDim.x) {
    double sg, cg, sb, cb;
    sincos(gamma[l], &sg, &cg);
    sincos(beta[l], &sb, &cb);
    const double2 one = make_double2(1.0, 0.0);
    const double2 ph = make_double2(cg, -sg), phc = make_double2(cg, sg);
    const double2 c = make_double2(cb, 0.0), ms = make_double2(0.0, -sb),
                  ps = make_double2(0.0, sb);
    T *t = table + 32 * l;
    put2x2<T>(t + 0, one, ph, ph, one);    // P
    put2x2<T>(t + 8, one, phc, phc, one);  // Pc
    put2x2<T>(t + 16, c, ms, ms, c);       // R
    put2x2<T>(t + 24, c, ps, ps, c);       // Rc
  }
  if (threadIdx.x == 0) {
    const double r2 = 0.70710678118654752440;
    T *t = table + 32 * p;
    t[0] = make_c<T>(r2, 0.0);  // H
    t[1] = make_c<T>(r2, 0.0);
    t[2] = make_c<T>(1.0, 0.0);  // Z
    t[3] = make_c<T>(-1.0, 0.0);
  }
}

// Block b fills network b % n_nets for angle set b / n_nets; the angles of
// set s start at angles + s * n_angles.
__global__ void k_fill(char *__restrict__ data, const double *__restrict__ angles,
                       const FillDesc *__restrict__ fills, int n_nets, int n_angles) {
  const int set = blockIdx.x / n_nets;
  const FillDesc f = fills[blockIdx.x % n_nets];
  const double *gamma = angles + (int64_t)set * n_angles + f.angle_off, *beta = gamma + f.p;
  if (f.table128 >= 0)
    fill_table<double2>((double2 *)(data + f.table128 + set * f.sstride128), gamma, beta, f.p);
  if (f.table64 >= 0)
    fill_table<float2>((float2 *)(data + f.table64 + set * f.sstride64), gamma, beta, f.p);
}

// Block s reduces angle set s: its scalar slots start scalar_sstride bytes
// after those of set s - 1, its results 2 n_cones + n_nets doubles after.
template <class T>
__global__ void k_reduce(const char *__restrict__ scalar_base, int64_t scalar_sstride,
                         const int *__restrict__ csb, const int *__restrict__ ncb,
                         const int *__restrict__ cns, int n_cones, int n_nets,
                         double *__restrict__ res_base) {
  const T *scalars = (const T *)(scalar_base + blockIdx.x * scalar_sstride);
  double *res = res_base + (int64_t)blockIdx.x * (2 * n_cones + n_nets);
  for (int c = threadIdx.x; c < n_cones; c += blockDim.x) {
    // the cone's slots split into cns[c] runs, one per slice (index
    // slicing); e_jk is the sum over slices of each run's product
    const int n_sl = cns[c], per = (csb[c + 1] - csb[c]) / n_sl;
    double sre = 0.0, sim = 0.0;
    for (int k = 0; k < n_sl; k++) {
      double re = 1.0, im = 0.0;
      for (int s = csb[c] + k * per; s < csb[c] + (k + 1) * per; s++) {
        const double2 z = to_d(scalars[s]);
        const double nr = re * z.x - im * z.y, ni = re * z.y + im * z.x;
        re = nr;
        im = ni;
      }
      if (n_sl == 1) {
        sre = re;
        sim = im;
      } else {
        sre += re;
        sim += im;
      }
    }
    res[c] = sre;
    res[n_cones + c] = sim;
  }
  __syncthreads();
  for (int n = threadIdx.x; n < n_nets; n += blockDim.x) {
    double sum = 0.0, comp = 0.0;
    for (int c = ncb[n]; c < ncb[n + 1]; c++) {
      const double x = res[c], t = sum + x;
      comp += (fabs(sum) >= fabs(x)) ? (sum - t) + x : (x - t) + sum;
      sum = t;
    }
    res[2 * n_cones + n] = 0.5 * (double)(ncb[n + 1] - ncb[n]) - 0.5 * (sum + comp);
  }
}

}  // namespace

// Grid of a wide launch: one wave per unit up to the blocks the device holds
// at once (all of them resident, so that the blocks of an XCD walk
// neighbouring units together and share their operand data in its L2), a
// multiple of the 8 XCDs.  Residency is queried once per kernel, LDS size and
// device.
template <class K>
int wide_grid(K kernel, size_t lds, uint32_t n_units, uint32_t units_per_block = kBlock / 64) {
  static std::mutex mu;
  static std::map<std::tuple<const void *, size_t, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  const auto key = std::make_tuple((const void *)kernel, lds, dev);
  int resident = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      resident = it->second;
    } else {
      int per_cu = 0, n_cu = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, lds) != hipSuccess ||
          hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        per_cu = n_cu = 0;
      resident = std::max(1, per_cu) * std::max(1, n_cu);
      cache[key] = resident;
    }
  }
  uint32_t b = n_units / units_per_block + (n_units % units_per_block ? 1u : 0u);
  if (b > (uint32_t)resident) b = (uint32_t)resident;
  if (b >= 8) b &= ~7u;
  return (int)(b ? b : 1);
}

// Launch with optional start/stop events attached to the dispatch itself:
// they time the kernel alone, without queueing or event-packet overhead.
#define QTN_LAUNCH_LDS(t0, t1, K, grid, block, lds, s, ...)                  \
  do {                                                                      \
    if (t0)                                                                 \
      hipExtLaunchKernelGGL(K, grid, block, lds, s, t0, t1, 0, __VA_ARGS__); \
    else                                                                    \
      hipLaunchKernelGGL(K, grid, block, lds, s, __VA_ARGS__);              \
  } while (0)
#define QTN_LAUNCH(t0, t1, K, grid, block, s, ...) \
  QTN_LAUNCH_LDS(t0, t1, K, grid, block, 0, s, __VA_ARGS__)

// Nothing to launch: the timing events still complete (zero duration).
inline hipError_t no_launch(hipEvent_t t0, hipEvent_t t1, hipStream_t s) {
  if (!t0) return hipSuccess;
  hipError_t e = hipEventRecord(t0, s);
  return e == hipSuccess ? hipEventRecord(t1, s) : e;
}

hipError_t launch_fill(int prec, void *data, const double *angles, const FillDesc *fills,
                       int n_nets, int n_angles, int n_sets, hipStream_t s) {
  (void)prec;
  hipLaunchKernelGGL(k_fill, dim3(n_nets * n_sets), dim3(64), 0, s, (char *)data, angles, fills,
                     n_nets, n_angles);
  return hipGetLastError();
}

hipError_t launch_block_groups(int prec, void *data, const DevGroup *groups, const DevOp *ops,
                               const int32_t *stab, const uint8_t *uperm, const int2 *ranges,
                               int range_base, int n_blocks, int n_sets, hipStream_t s,
                               hipEvent_t t0, hipEvent_t t1) {
  (void)prec;
  if (n_blocks <= 0 || n_sets <= 0) return no_launch(t0, t1, s);
  QTN_LAUNCH(t0, t1, k_block_groups, dim3(n_blocks * n_sets), dim3(kBlock), s, (char *)data,
             groups, ops, stab, uperm, ranges, range_base, n_blocks);
  return hipGetLastError();
}

template <class T, bool CVT>
void launch_wide_t(const DevGroup &hg, uint32_t units, char *d, const DevGroup *groups,
                   const DevOp *ops, const int32_t *stab, const uint8_t *uperm, int group,
                   uint32_t n_sets, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  if (hg.variant == kVarStream) {
    const size_t lds = (size_t)hg.n_ops * 64 * sizeof(uint32_t);
    const int nb = wide_grid(k_wide_stream<T, CVT>, lds, units);
    QTN_LAUNCH_LDS(t0, t1, (k_wide_stream<T, CVT>), dim3(nb), dim3(kBlock), lds, s, d, groups, ops,
                   stab, uperm, group, n_sets);
  } else if (hg.variant == kVarCell) {
    const size_t lds = cell_lds_words(hg.n_ops, hg.rls) * sizeof(uint32_t);
#define QTN_CELL_LAUNCH(CB, SL)                                                                  \
  do {                                                                                           \
    const int nb = wide_grid(k_wide_cells<T, CVT, CB, SL>, lds, units);                         \
    QTN_LAUNCH_LDS(t0, t1, (k_wide_cells<T, CVT, CB, SL>), dim3(nb), dim3(kBlock), lds, s, d,   \
                   groups, ops, stab, uperm, group, n_sets);                                      \
  } while (0)
    if (hg.rls == 2 && hg.sl == 0) QTN_CELL_LAUNCH(2, 0);
    else if (hg.rls == 2 && hg.sl == 1) QTN_CELL_LAUNCH(2, 1);
    else if (hg.rls == 2) QTN_CELL_LAUNCH(2, 2);
    else if (hg.rls == 3 && hg.sl == 0) QTN_CELL_LAUNCH(3, 0);
    else if (hg.rls == 3 && hg.sl == 1) QTN_CELL_LAUNCH(3, 1);
    else if (hg.rls == 3) QTN_CELL_LAUNCH(3, 2);
    else if (hg.sl == 0) QTN_CELL_LAUNCH(4, 0);
    else if (hg.sl == 1) QTN_CELL_LAUNCH(4, 1);
    else QTN_CELL_LAUNCH(4, 2);
#undef QTN_CELL_LAUNCH
  } else {
    const int nb = wide_grid(k_wide_generic<T, CVT>, 0, units);
    QTN_LAUNCH(t0, t1, (k_wide_generic<T, CVT>), dim3(nb), dim3(kBlock), s, d, groups, ops, stab,
               uperm, group, n_sets);
  }
}

hipError_t launch_wide_group(const DevGroup &hg, void *data, const DevGroup *groups,
                             const DevOp *ops, const int32_t *stab, const uint8_t *uperm,
                             int group, int n_sets, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  const uint32_t n_units = hg.n_units;
  // the unit walk needs the flat unit count plus the grid's waves below 2^32
  if (n_sets <= 0 || (uint64_t)n_units * (uint64_t)n_sets > 0x7FFFFFFFull) return hipErrorInvalidValue;
  if ((hg.variant == kVarStream || hg.variant == kVarCell) &&
      (hg.n_ops < 1 || hg.n_ops > kStreamMaxOps))
    return hipErrorInvalidValue;
  if (hg.variant == kVarCell && (hg.rls < kCellMinCB || hg.rls > kCellMaxCB || hg.n_ops > 64 ||
                                 hg.sl > kCellMaxSerial || hg.sl > hg.rls ||
                                 cell_lds_words(hg.n_ops, hg.rls) > kCellMaxLdsWords))
    return hipErrorInvalidValue;
  const uint32_t ns = (uint32_t)n_sets, units = n_units * ns;
  char *d = (char *)data;
  const bool cvt = hg.cvt != 0;
  if (hg.variant == kVarMfma) {
    // a unit is one tile of the whole block
#define QTN_MM_LAUNCH3(T, C, NCB)                                                             \
  do {                                                                                       \
    const int nb = wide_grid(k_wide_mfma<T, C, NCB>, 0, units, 1);                           \
    QTN_LAUNCH(t0, t1, (k_wide_mfma<T, C, NCB>), dim3(nb), dim3(kBlock), s, d, groups, ops,   \
               stab, uperm, group, ns);                                                      \
  } while (0)
#define QTN_MM_LAUNCH(T, C)                                   \
  do {                                                        \
    if (hg.rls == 1) QTN_MM_LAUNCH3(T, C, 1);                 \
    else if (hg.rls == 2) QTN_MM_LAUNCH3(T, C, 2);            \
    else QTN_MM_LAUNCH3(T, C, 4);                             \
  } while (0)
    if (hg.prec == kPrecC128 && !cvt) QTN_MM_LAUNCH(double2, false);
    else if (hg.prec == kPrecC128) QTN_MM_LAUNCH(double2, true);
    else if (!cvt) QTN_MM_LAUNCH(float2, false);
    else QTN_MM_LAUNCH(float2, true);
#undef QTN_MM_LAUNCH
#undef QTN_MM_LAUNCH3
    return hipGetLastError();
  }
  if (hg.prec == kPrecC128 && !cvt)
    launch_wide_t<double2, false>(hg, units, d, groups, ops, stab, uperm, group, ns, s, t0, t1);
  else if (hg.prec == kPrecC128)
    launch_wide_t<double2, true>(hg, units, d, groups, ops, stab, uperm, group, ns, s, t0, t1);
  else if (!cvt)
    launch_wide_t<float2, false>(hg, units, d, groups, ops, stab, uperm, group, ns, s, t0, t1);
  else
    launch_wide_t<float2, true>(hg, units, d, groups, ops, stab, uperm, group, ns, s, t0, t1);
  return hipGetLastError();
}

hipError_t launch_persistent(int prec, void *data, const DevGroup *groups, const DevOp *ops,
                             const int32_t *stab, const uint8_t *uperm, const int4 *items,
                             const int *step_begin, int n_steps, uint32_t *ctl, int n_ctl,
                             int n_blocks, uint32_t spin_limit, hipStream_t s, hipEvent_t t0,
                             hipEvent_t t1) {
  (void)prec;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, s, ctl, n_ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (n_steps <= 0) return no_launch(t0, t1, s);
  QTN_LAUNCH(t0, t1, k_persistent, dim3(n_blocks), dim3(kBlock), s, (char *)data, groups, ops,
             stab, uperm, items, step_begin, n_steps, ctl, spin_limit);
  return hipGetLastError();
}

hipError_t launch_dataflow(void *data, const DevGroup *groups, const DevOp *ops,
                           const int32_t *stab, const uint8_t *uperm, const int4 *items,
                           int n_items, int n_init, const int *item_task, const int *task_next,
                           const int *task_first, const int *task_need, uint32_t *queue,
                           uint32_t *ctl, int n_ctl, int n_blocks, uint32_t spin_limit,
                           hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  const int span = n_ctl > n_items ? n_ctl : n_items;
  hipLaunchKernelGGL(k_queue_reset, dim3((span + 255) / 256), dim3(256), 0, s, ctl, n_ctl, queue,
                     n_items, n_init);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (n_items <= 0) return no_launch(t0, t1, s);
  QTN_LAUNCH(t0, t1, k_dataflow, dim3(n_blocks), dim3(kBlock), s, (char *)data, groups, ops, stab,
             uperm, items, n_items, item_task, task_next, task_first, task_need, queue, ctl,
             spin_limit);
  return hipGetLastError();
}

int persistent_blocks(int prec, int n_cu) {
  (void)prec;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent, kBlock, 0);
  if (e != hipSuccess || per_cu < 1) return 0;
  return per_cu * n_cu;
}

hipError_t launch_reduce(int prec, const void *data, int64_t scalar_off, int64_t scalar_sstride,
                         const int *csb, const int *ncb, const int *cns, int n_cones, int n_nets,
                         int n_sets, double *res, hipStream_t s) {
  const char *sc = (const char *)data + scalar_off;
  if (prec == kPrecC64)
    hipLaunchKernelGGL(k_reduce<float2>, dim3(n_sets), dim3(256), 0, s, sc, scalar_sstride, csb,
                       ncb, cns, n_cones, n_nets, res);
  else
    hipLaunchKernelGGL(k_reduce<double2>, dim3(n_sets), dim3(256), 0, s, sc, scalar_sstride, csb,
                       ncb, cns, n_cones, n_nets, res);
  return hipGetLastError();
}

// Descriptor scratch of the allocation-free single-bucket entry point: a
// file-scope device array, one copy per GPU, held until the process ends.
// In host code `scratch` names a host-side stand-in; kernels get the device
// address looked up below.
static __device__ __align__(256) char scratch[kScratchBytes];

hipError_t scratch_address(void **out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    // once per device, with that device current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

}  // namespace qtn
