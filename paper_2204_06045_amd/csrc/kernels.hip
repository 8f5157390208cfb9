// HIP kernels for gfx950 (CDNA4): bucket contraction over fused groups.
//
// Bucket elimination (arXiv 2204.06045, Sec. II-B) contracts a bucket by
// multiplying its tensors over the union of their binary indices and summing
// the bucket index; merged indices (Sec. II-C) sum several nested buckets in
// one pass.  A fused group here is such a chain of L buckets: with the union
// index I (bit 0 = first bucket index), level-l operands are multiplied in
// after bits 0..l-1 have been summed, and the group writes out[I >> L].
//
// Thread mapping (wave64): a wave evaluates one unit of 2^(RG+6) union points;
// bits [0, RG) are held in registers by each lane, bits [RG, RG+6) select the
// lane, the rest select the unit.  Summed bits in registers are added in
// registers; summed lane bits are added with cross-lane butterflies.  Operand
// t is read at pext(I, mask_t), computed from the contiguous runs of the mask.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace qtn {
namespace {

constexpr int RG = 2;  // register bits per lane
constexpr int kBlock = 256;

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

// pext over the operand's mask, from its runs (uniform per wave).
__device__ __forceinline__ uint32_t pext_runs(uint32_t x, const DevOp &o) {
  uint32_t r = 0;
  const int nr = o.nruns;
  for (int i = 0; i < nr; i++)
    r |= ((x >> o.rs[i]) & (uint32_t)((1ull << o.rl[i]) - 1ull)) << o.rd[i];
  return r;
}

// pext of a register-field value x < 2^RG over the low RG mask bits.
__device__ __forceinline__ uint32_t pext_reg(uint32_t x, uint32_t m) {
  uint32_t r = 0, d = 0;
#pragma unroll
  for (int b = 0; b < RG; b++)
    if ((m >> b) & 1u) {
      r |= ((x >> b) & 1u) << d;
      d++;
    }
  return r;
}

template <class T>
__device__ __forceinline__ void eval_unit(const DevGroup &G, const DevOp *__restrict__ ops,
                                          T *__restrict__ data, uint32_t u, int lane) {
  constexpr int NR = 1 << RG;
  const uint32_t I0 = (u << (RG + 6)) | ((uint32_t)lane << RG);
  const int L = G.L;
  const DevOp *gops = ops + G.op_begin;
  T v[NR];

  // level 0: product of the first bucket's tensors at the NR register points
  {
    const DevOp &o = gops[0];
    const uint32_t base = pext_runs(I0, o);
    const T *src = data + o.off;
#pragma unroll
    for (int r = 0; r < NR; r++) v[r] = src[base + pext_reg(r, o.mask)];
  }
  int k = 1;
  for (; k < G.level_end[0]; k++) {
    const DevOp &o = gops[k];
    const uint32_t base = pext_runs(I0, o);
    const T *src = data + o.off;
#pragma unroll
    for (int r = 0; r < NR; r++) v[r] = cmul(v[r], src[base + pext_reg(r, o.mask)]);
  }

  // summed bits held in registers
#pragma unroll
  for (int s = 0; s < RG; s++) {
    if (s < L) {
#pragma unroll
      for (int r = 0; r < (NR >> (s + 1)); r++) v[r] = cadd(v[2 * r], v[2 * r + 1]);
      if (s + 1 < L) {
        for (; k < G.level_end[s + 1]; k++) {
          const DevOp &o = gops[k];
          const uint32_t base = pext_runs(I0, o);
          const T *src = data + o.off;
#pragma unroll
          for (int r = 0; r < (NR >> (s + 1)); r++)
            v[r] = cmul(v[r], src[base + pext_reg((uint32_t)r << (s + 1), o.mask)]);
        }
      }
    }
  }

  T *out = data + G.out_off;
  const uint32_t nout = 1u << (G.w - L);
  if (L <= RG) {
    const uint32_t ob = I0 >> L;
#pragma unroll
    for (int r = 0; r < NR; r++)
      if (r < (NR >> L) && ob + r < nout) out[ob + r] = v[r];
    return;
  }

  // summed bits spread over lanes: butterflies, then the next level's tensors
  T acc = v[0];
  for (int s = RG; s < L; s++) {
    acc = cadd(acc, shfl_xor2(acc, 1 << (s - RG)));
    if (s + 1 < L) {
      for (; k < G.level_end[s + 1]; k++) {
        const DevOp &o = gops[k];
        acc = cmul(acc, data[o.off + pext_runs(I0, o)]);
      }
    }
  }
  if ((lane & ((1 << (L - RG)) - 1)) == 0) {
    const uint32_t o = I0 >> L;
    if (o < nout) out[o] = acc;
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_block_groups(T *__restrict__ data,
                                                         const DevGroup *__restrict__ groups,
                                                         const DevOp *__restrict__ ops,
                                                         const int2 *__restrict__ ranges,
                                                         int range_base) {
  const int2 rg = ranges[range_base + blockIdx.x];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  for (int g = rg.x; g < rg.y; g++) {
    const DevGroup G = groups[g];
    for (uint32_t u = wave; u < G.n_units; u += nw) eval_unit<T>(G, ops, data, u, lane);
    __syncthreads();  // this group's output is read by the next ones
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_wide_group(T *__restrict__ data,
                                                       const DevGroup *__restrict__ groups,
                                                       const DevOp *__restrict__ ops, int gid) {
  const DevGroup G = groups[gid];
  const int lane = threadIdx.x & 63;
  const uint32_t nb = gridDim.x, b = blockIdx.x;
  // Blocks are dealt round-robin to the 8 XCDs; renumber them so that each
  // XCD walks one contiguous slice of the union space (its own L2).
  const uint32_t lb = (nb % 8u == 0u) ? (b % 8u) * (nb / 8u) + b / 8u : b;
  const uint32_t per = (G.n_units + nb - 1) / nb;
  const uint32_t ub = lb * per;
  const uint32_t ue = min(G.n_units, ub + per);
  const uint32_t nw = blockDim.x >> 6;
  for (uint32_t u = ub + (threadIdx.x >> 6); u < ue; u += nw) eval_unit<T>(G, ops, data, u, lane);
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
__global__ void k_fill(T *__restrict__ data, const double *__restrict__ angles,
                       const FillDesc *__restrict__ fills) {
  const FillDesc f = fills[blockIdx.x];
  T *table = data + f.table_off;
  const double *gamma = angles + f.angle_off, *beta = gamma + f.p;
  for (int l = threadIdx.x; l < f.p; l += blockDim.x) {
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
    T *t = table + 32 * f.p;
    t[0] = make_c<T>(r2, 0.0);  // H
    t[1] = make_c<T>(r2, 0.0);
    t[2] = make_c<T>(1.0, 0.0);  // Z
    t[3] = make_c<T>(-1.0, 0.0);
  }
}

template <class T>
__global__ void k_reduce(const T *__restrict__ scalars, const int *__restrict__ csb,
                         const int *__restrict__ ncb, int n_cones, int n_nets,
                         double *__restrict__ res) {
  for (int c = threadIdx.x; c < n_cones; c += blockDim.x) {
    double re = 1.0, im = 0.0;
    for (int s = csb[c]; s < csb[c + 1]; s++) {
      const double2 z = to_d(scalars[s]);
      const double nr = re * z.x - im * z.y, ni = re * z.y + im * z.x;
      re = nr;
      im = ni;
    }
    res[c] = re;
    res[n_cones + c] = im;
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

int wide_blocks(uint32_t n_units) {
  const uint32_t waves = kBlock / 64;
  uint32_t b = (n_units + waves - 1) / waves;
  if (b > 2048) b = 2048;
  if (b >= 8) b &= ~7u;
  return (int)(b ? b : 1);
}

hipError_t launch_fill(int prec, void *data, const double *angles, const FillDesc *fills,
                       int n_nets, hipStream_t s) {
  if (prec == kPrecC128)
    hipLaunchKernelGGL(k_fill<double2>, dim3(n_nets), dim3(64), 0, s, (double2 *)data, angles,
                       fills);
  else
    hipLaunchKernelGGL(k_fill<float2>, dim3(n_nets), dim3(64), 0, s, (float2 *)data, angles,
                       fills);
  return hipGetLastError();
}

hipError_t launch_block_groups(int prec, void *data, const DevGroup *groups, const DevOp *ops,
                               const int2 *ranges, int range_base, int n_blocks,
                               hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  if (prec == kPrecC128)
    hipLaunchKernelGGL(k_block_groups<double2>, dim3(n_blocks), dim3(kBlock), 0, s,
                       (double2 *)data, groups, ops, ranges, range_base);
  else
    hipLaunchKernelGGL(k_block_groups<float2>, dim3(n_blocks), dim3(kBlock), 0, s,
                       (float2 *)data, groups, ops, ranges, range_base);
  return hipGetLastError();
}

hipError_t launch_wide_group(int prec, void *data, const DevGroup *groups, const DevOp *ops,
                             int group, uint32_t n_units, hipStream_t s) {
  const int nb = wide_blocks(n_units);
  if (prec == kPrecC128)
    hipLaunchKernelGGL(k_wide_group<double2>, dim3(nb), dim3(kBlock), 0, s, (double2 *)data,
                       groups, ops, group);
  else
    hipLaunchKernelGGL(k_wide_group<float2>, dim3(nb), dim3(kBlock), 0, s, (float2 *)data,
                       groups, ops, group);
  return hipGetLastError();
}

hipError_t launch_reduce(int prec, const void *data, int64_t scalar_off, const int *csb,
                         const int *ncb, int n_cones, int n_nets, double *res, hipStream_t s) {
  if (prec == kPrecC128)
    hipLaunchKernelGGL(k_reduce<double2>, dim3(1), dim3(256), 0, s,
                       (const double2 *)data + scalar_off, csb, ncb, n_cones, n_nets, res);
  else
    hipLaunchKernelGGL(k_reduce<float2>, dim3(1), dim3(256), 0, s,
                       (const float2 *)data + scalar_off, csb, ncb, n_cones, n_nets, res);
  return hipGetLastError();
}

}  // namespace qtn
