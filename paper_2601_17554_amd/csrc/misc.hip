// Small kernels around the dense products: batch sanitising and the attention work list, the
// second layer of the output heads with the argmax and decode, and a plain copy.
#include "common.h"
#include "kernels.h"

namespace mlpf {

// ---------------------------------------------------------------------------------------------
// Work list. One workgroup reads the caller's row offsets, clamps them into [0, total_rows] (and
// the valid counts into the event's span and max_seqlen), and lists attention work items
// (event, query tile, head) with events in order of decreasing key count. Workgroups are
// dispatched roughly in launch order, so the longest items start first (longest-processing-time
// order), which keeps the tail of a varlen batch short. Items of one event are ordered query
// tile-major, head-minor: with a multiple of 8 heads, consecutive items go to the 8 XCDs in turn
// and each XCD's L2 then serves one head's K and V.
constexpr int kWlThreads = 1024;
constexpr int kWlBuckets = 8192 / 64 + 2;  // cost buckets: ceil(n / 64) in 0..128

__global__ __launch_bounds__(kWlThreads) void worklist_kernel(const WorklistArgs p) {
  __shared__ int s_items[kWlBuckets];   // items per bucket
  __shared__ int s_cursor[kWlBuckets];  // next free item slot per bucket
  __shared__ int s_total;
  const int tid = threadIdx.x;
  for (int b = tid; b < kWlBuckets; b += kWlThreads) s_items[b] = 0;
  __syncthreads();

  const int T = p.total_rows;
  for (int e = tid; e < p.n_events; e += kWlThreads) {
    const int s = min(max(p.row_start[e], 0), T);
    const int en = min(max(p.row_start[e + 1], s), T);
    int n = en - s;
    if (p.n_valid) n = min(max(p.n_valid[e], 0), n);
    n = min(n, p.max_seqlen);
    p.ev_start[e] = s;
    p.ev_n[e] = n;
    const int items = ((n + p.q_tile - 1) / p.q_tile) * p.n_heads;
    atomicAdd(&s_items[(n + 63) / 64], items);
  }
  if (tid == 0) *p.n_rows = p.n_events > 0 ? min(max(p.row_start[p.n_events], 0), T) : 0;
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int b = kWlBuckets - 1; b >= 0; --b) {
      s_cursor[b] = acc;
      acc += s_items[b];
    }
    s_total = min(acc, p.cap_items);
    *p.n_items = s_total;
  }
  __syncthreads();
  // The writes to ev_start/ev_n above are read back below by other threads of this workgroup.
  __threadfence_block();

  // Each event reserves its slot range (order inside a bucket is irrelevant to the results).
  // Offsets are kept in the items array's tail-free region via a second pass below.
  for (int e0 = 0; e0 < p.n_events; e0 += kWlThreads) {
    __shared__ int s_off[kWlThreads];
    const int e = e0 + tid;
    int n = 0;
    if (e < p.n_events) {
      n = p.ev_n[e];
      const int items = ((n + p.q_tile - 1) / p.q_tile) * p.n_heads;
      s_off[tid] = atomicAdd(&s_cursor[(n + 63) / 64], items);
    }
    __syncthreads();
    const int cnt = min(kWlThreads, p.n_events - e0);
    for (int j = 0; j < cnt; ++j) {
      const int ej = e0 + j;
      const int nj = p.ev_n[ej];
      const int items = ((nj + p.q_tile - 1) / p.q_tile) * p.n_heads;
      const int off = s_off[j];
      for (int it = tid; it < items; it += kWlThreads) {
        const int slot = off + it;
        if (slot < p.cap_items) {
          const int qt = it / p.n_heads, hd = it % p.n_heads;
          p.items[2 * slot] = ej;
          p.items[2 * slot + 1] = (qt << 8) | hd;
        }
      }
    }
    __syncthreads();
  }
}

hipError_t launch_worklist(const WorklistArgs& p, hipStream_t s) {
  hipLaunchKernelGGL(worklist_kernel, dim3(1), dim3(kWlThreads), 0, s, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// The class of a row from its six classification outputs (Sec. 5.3 inference rule). binary = 0:
// argmax of the six logits, class 0 = no particle, the lowest index on exact ties. binary = 1:
// output 0 is the binary "is a particle" logit, kept when sigmoid > 0.5, i.e. logit > 0; the class
// is then 1 + the argmax of the five particle-type logits (lowest index on ties), else 0.
__device__ __forceinline__ int decide_class(const float (&acc)[11], int binary) {
  if (binary) {
    if (!(acc[0] > 0.f)) return 0;
    int best = 1;
#pragma unroll
    for (int c = 2; c < 6; ++c)
      if (acc[c] > acc[best]) best = c;
    return best;
  }
  int best = 0;
#pragma unroll
  for (int c = 1; c < 6; ++c)
    if (acc[c] > acc[best]) best = c;
  return best;
}

// Second layer of the heads (block diagonal [nh d] -> 11), class rule, decode. One wave per row:
// lanes read the row's hidden activations coalesced, each keeps 11 partial dot products, and the
// wave reduces them. NH = 5: output columns cls 0..5, pT 6, eta 7, phi 8..9, E 10 read heads
// 0, 1, 2, 3, 4; NH = 6: binary 0 and pid 1..5 read heads 0 and 1, the rest heads 2..5.
template <int NH>
__device__ constexpr int head_of_col(int c) {
  if (c < 6) return (NH == 6 && c > 0) ? 1 : 0;
  const int r = c == 6 ? 0 : c == 7 ? 1 : c <= 9 ? 2 : 3;  // pT, eta, phi (sin, cos), E
  return NH - 4 + r;
}

template <class S, int NH>
__global__ __launch_bounds__(256) void heads2_kernel(const Heads2Args p) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  int M = p.rows;
  if (p.m_dev) M = min(M, max(*p.m_dev, 0));
  if (row >= M) return;
  const S* u = (const S*)p.uh + (int64_t)row * NH * p.d;
  float acc[11];
#pragma unroll
  for (int c = 0; c < 11; ++c) acc[c] = 0.f;
  for (int j = lane; j < p.d; j += 64) {
    const float* w = p.w2 + j * 11;
    float uk[NH];
#pragma unroll
    for (int k = 0; k < NH; ++k) uk[k] = (float)u[k * p.d + j];
#pragma unroll
    for (int c = 0; c < 11; ++c) acc[c] += uk[head_of_col<NH>(c)] * w[c];
  }
#pragma unroll
  for (int c = 0; c < 11; ++c) acc[c] = wave_sum(acc[c]) + p.b2[c];
  if (lane == 0) {
    const int best = decide_class(acc, p.binary);
    float* lg = p.logits + (int64_t)row * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) lg[c] = acc[c];
    float* rg = p.reg + (int64_t)row * 5;
#pragma unroll
    for (int c = 0; c < 5; ++c) rg[c] = acc[6 + c];
    p.cls[row] = best;
    if (p.prim && p.decoded) {
      float* dd = p.decoded + (int64_t)row * 4;
      dd[0] = p.prim[2 * row] * expf(acc[6]);
      dd[1] = acc[7];
      dd[2] = atan2f(acc[8], acc[9]);
      dd[3] = p.prim[2 * row + 1] * expf(acc[10]);
    }
  }
}

hipError_t launch_heads2(Prec prec, const Heads2Args& p, hipStream_t s) {
  const int grid = (p.rows + 3) / 4;
  if (grid == 0) return hipSuccess;
  if (prec == P_F32 && p.heads6)
    hipLaunchKernelGGL((heads2_kernel<float, 6>), dim3(grid), dim3(256), 0, s, p);
  else if (prec == P_F32)
    hipLaunchKernelGGL((heads2_kernel<float, 5>), dim3(grid), dim3(256), 0, s, p);
  else if (p.heads6)
    hipLaunchKernelGGL((heads2_kernel<__bf16, 6>), dim3(grid), dim3(256), 0, s, p);
  else
    hipLaunchKernelGGL((heads2_kernel<__bf16, 5>), dim3(grid), dim3(256), 0, s, p);
  return hipGetLastError();
}

// Output stage after the fused head GEMM: one thread per row adds b2 to the 11 second-layer sums
// that the GEMM epilogue wrote, then argmax and decode as above.
__global__ __launch_bounds__(256) void heads_finish_kernel(const Heads2Args p) {
  const int row = blockIdx.x * 256 + threadIdx.x;
  int M = p.rows;
  if (p.m_dev) M = min(M, max(*p.m_dev, 0));
  if (row >= M) return;
  const float* u = (const float*)p.uh + (int64_t)row * 11;
  float acc[11];
#pragma unroll
  for (int c = 0; c < 11; ++c) acc[c] = u[c] + p.b2[c];
  const int best = decide_class(acc, p.binary);
  float* lg = p.logits + (int64_t)row * 6;
#pragma unroll
  for (int c = 0; c < 6; ++c) lg[c] = acc[c];
  float* rg = p.reg + (int64_t)row * 5;
#pragma unroll
  for (int c = 0; c < 5; ++c) rg[c] = acc[6 + c];
  p.cls[row] = best;
  if (p.prim && p.decoded) {
    float* dd = p.decoded + (int64_t)row * 4;
    dd[0] = p.prim[2 * row] * expf(acc[6]);
    dd[1] = acc[7];
    dd[2] = atan2f(acc[8], acc[9]);
    dd[3] = p.prim[2 * row + 1] * expf(acc[10]);
  }
}

hipError_t launch_heads_finish(const Heads2Args& p, hipStream_t s) {
  const int grid = (p.rows + 255) / 256;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(heads_finish_kernel, dim3(grid), dim3(256), 0, s, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// LayerNorm of FP32 rows into the operand type of the next product (pre-LN transformer block):
// FP32, BF16, or FP8 E4M3 after multiplying by out_scale (the inverse per-tensor scale).
// One wave per row; the row stays in registers (d <= 1024: up to 4 float4 per lane), statistics
// in FP32 with two passes over the registers (mean, then mean squared deviation = biased
// variance).
template <class S, int V, int XB>  // V = 4-element chunks per lane, XB = bytes per input element
__global__ __launch_bounds__(256) void layernorm_kernel(const LayerNormArgs p) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  int M = p.rows;
  if (p.m_dev) M = min(M, max(*p.m_dev, 0));
  if (row >= M) return;
  f32x4 v[V];
  float s = 0.f;
#pragma unroll
  for (int t = 0; t < V; ++t) {
    const int c = lane + 64 * t;
    v[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (4 * c < p.d) {
      if constexpr (XB == 4) {
        v[t] = ((const f32x4*)((const float*)p.x + (int64_t)row * p.d))[c];
      } else {
        const u32x2 w = ((const u32x2*)((const __bf16*)p.x + (int64_t)row * p.d))[c];
        v[t] = f32x4{__uint_as_float(w[0] << 16), __uint_as_float(w[0] & 0xffff0000u),
                     __uint_as_float(w[1] << 16), __uint_as_float(w[1] & 0xffff0000u)};
      }
    }
    s = add_nc(s, ln_sum4(v[t][0], v[t][1], v[t][2], v[t][3]));
  }
  const float mu = ln_mean(wave_sum(s), p.d);
  float q = 0.f;
#pragma unroll
  for (int t = 0; t < V; ++t) {
    const int c = lane + 64 * t;
    if (4 * c < p.d) q = add_nc(q, ln_sq4(v[t][0], v[t][1], v[t][2], v[t][3], mu));
  }
  const float rs = ln_rstd(wave_sum(q), p.d, p.eps);
  S* y = (S*)p.y + (int64_t)row * p.d;
  float amax = 0.f;
#pragma unroll
  for (int t = 0; t < V; ++t) {
    const int c = lane + 64 * t;
    if (4 * c >= p.d) continue;
    const f32x4 g = ((const f32x4*)p.gamma)[c], b = ((const f32x4*)p.beta)[c];
    const float o0 = ln_out(v[t][0], mu, rs, g[0], b[0]);
    const float o1 = ln_out(v[t][1], mu, rs, g[1], b[1]);
    const float o2 = ln_out(v[t][2], mu, rs, g[2], b[2]);
    const float o3 = ln_out(v[t][3], mu, rs, g[3], b[3]);
    amax = fmaxf(amax, fmaxf(fmaxf(fabsf(o0), fabsf(o1)), fmaxf(fabsf(o2), fabsf(o3))));
    if constexpr (sizeof(S) == 4)
      *(f32x4*)(y + 4 * c) = f32x4{o0, o1, o2, o3};
    else if constexpr (sizeof(S) == 2)
      *(u32x2*)(y + 4 * c) = pack_bf16x4(o0, o1, o2, o3);
    else
      *(uint32_t*)(y + 4 * c) = pack_fp8x4(o0 * p.out_scale, o1 * p.out_scale, o2 * p.out_scale,
                                           o3 * p.out_scale);
  }
  if (p.amax) {
    amax = wave_max(amax);
    if (lane == 0) atomic_max_nonneg(p.amax, amax);
  }
}

template <class S>
hipError_t launch_ln_t(const LayerNormArgs& p, hipStream_t s) {
  const int grid = (p.rows + 3) / 4;
  const int v = (p.d + 255) / 256;
  if (p.x_bf16) {
    if (v <= 1)
      hipLaunchKernelGGL((layernorm_kernel<S, 1, 2>), dim3(grid), dim3(256), 0, s, p);
    else if (v <= 2)
      hipLaunchKernelGGL((layernorm_kernel<S, 2, 2>), dim3(grid), dim3(256), 0, s, p);
    else
      hipLaunchKernelGGL((layernorm_kernel<S, 4, 2>), dim3(grid), dim3(256), 0, s, p);
  } else {
    if (v <= 1)
      hipLaunchKernelGGL((layernorm_kernel<S, 1, 4>), dim3(grid), dim3(256), 0, s, p);
    else if (v <= 2)
      hipLaunchKernelGGL((layernorm_kernel<S, 2, 4>), dim3(grid), dim3(256), 0, s, p);
    else
      hipLaunchKernelGGL((layernorm_kernel<S, 4, 4>), dim3(grid), dim3(256), 0, s, p);
  }
  return hipGetLastError();
}

hipError_t launch_layernorm(Prec prec, const LayerNormArgs& p, hipStream_t s) {
  if (p.rows <= 0) return hipSuccess;
  if (p.d % 4 != 0 || p.d > 1024) return hipErrorInvalidValue;
  if (prec == P_F32) return launch_ln_t<float>(p, s);
  if (prec == P_BF16) return launch_ln_t<__bf16>(p, s);
  return launch_ln_t<uint8_t>(p, s);
}

// ---------------------------------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(256) void scale_kernel(S* dst, const S* src, int64_t n, float scale) {
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    dst[i] = (S)((float)src[i] * scale);
}

hipError_t launch_scale(Prec prec, void* dst, const void* src, int64_t n, float scale,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t grid = (n + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (prec == P_F32)
    hipLaunchKernelGGL(scale_kernel<float>, dim3((unsigned)grid), dim3(256), 0, s, (float*)dst,
                       (const float*)src, n, scale);
  else
    hipLaunchKernelGGL(scale_kernel<__bf16>, dim3((unsigned)grid), dim3(256), 0, s, (__bf16*)dst,
                       (const __bf16*)src, n, scale);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void copy_f32_kernel(float* dst, const float* src, int64_t n) {
  const int64_t n4 = n / 4;
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n4; i += (int64_t)gridDim.x * 256)
    ((f32x4*)dst)[i] = ((const f32x4*)src)[i];
  for (int64_t i = n4 * 4 + blockIdx.x * 256LL + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    dst[i] = src[i];
}

// One wave per row: 16-byte chunks of alt's row replace h's when the row is not a track.
__global__ __launch_bounds__(256) void select_rows_kernel(char* h, const char* alt, const float* x,
                                                          int F, int rows, const int32_t* m_dev,
                                                          int row_bytes) {
  int M = rows;
  if (m_dev) M = min(M, max(*m_dev, 0));
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= M) return;
  if (x[(int64_t)row * F] > 0.5f) return;  // a track keeps the track embedding
  const int64_t base = (int64_t)row * row_bytes;
  for (int o = (threadIdx.x & 63) * 16; o < row_bytes; o += 64 * 16)
    *(u32x4*)(h + base + o) = *(const u32x4*)(alt + base + o);
}

hipError_t launch_select_rows(void* h, const void* alt, const float* x, int n_features, int rows,
                              const int32_t* m_dev, int row_bytes, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  if (row_bytes % 16 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(select_rows_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, (char*)h,
                     (const char*)alt, x, n_features, rows, m_dev, row_bytes);
  return hipGetLastError();
}

hipError_t launch_copy_f32(float* dst, const float* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t grid = (n / 4 + 255) / 256;
  if (grid < 1) grid = 1;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(copy_f32_kernel, dim3((unsigned)grid), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

}  // namespace mlpf
