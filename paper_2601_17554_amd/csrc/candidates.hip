// Particle candidates per event (paper Sec. 5.3, inference rule; Sec. 8, the reconstruction
// module's output): every valid element whose predicted class is not 0 ("no particle") becomes a
// candidate with its class and decoded four-momentum, in element order within its event, events
// in order. Three launches: per-event counts (one workgroup per event), one exclusive scan over the
// events (one workgroup), per-event ordered writes (one workgroup per event, ballot prefix sums
// within a wave, wave totals through LDS). The batch description is clamped as in every other
// kernel of the library (row ranges into [0, total_rows], valid counts to the range and to
// max_seqlen).
#include "candidates.h"

namespace mlpf {

namespace {

constexpr int kCountThreads = 256;
constexpr int kScanThreads = 1024;

struct Range {
  int start, n;
};

__device__ __forceinline__ Range event_range(const CandArgs& p, int e) {
  const int T = p.total_rows;
  const int s = min(max(p.row_start[e], 0), T);
  const int en = min(max(p.row_start[e + 1], s), T);
  int n = en - s;
  if (p.n_valid) n = min(max(p.n_valid[e], 0), n);
  n = min(n, p.max_seqlen);
  return {s, n};
}

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// offsets[e + 1] = number of candidates of event e.
__global__ __launch_bounds__(kCountThreads) void cand_count_kernel(const CandArgs p) {
  __shared__ int part[kCountThreads / 64];
  const int e = blockIdx.x;
  const Range r = event_range(p, e);
  int c = 0;
  for (int i = threadIdx.x; i < r.n; i += kCountThreads) c += p.cls[r.start + i] != 0;
  c = wave_sum_i(c);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
#pragma unroll
    for (int w = 0; w < kCountThreads / 64; ++w) t += part[w];
    p.offsets[e + 1] = t;
  }
}

// In place: offsets[0] = 0, offsets[e + 1] = sum of the counts of events 0..e (one workgroup).
__global__ __launch_bounds__(kScanThreads) void cand_scan_kernel(const CandArgs p) {
  __shared__ int wtot[kScanThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) p.offsets[0] = 0;
  int carry = 0;
  for (int base = 0; base < p.n_events; base += kScanThreads) {
    const int i = base + tid;
    int v = i < p.n_events ? p.offsets[i + 1] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(v, o, 64);
      if (lane >= o) v += t;
    }
    if (lane == 63) wtot[wave] = v;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
      before += w < wave ? wtot[w] : 0;
      all += wtot[w];
    }
    if (i < p.n_events) p.offsets[i + 1] = carry + before + v;
    carry += all;
    __syncthreads();  // wtot is rewritten by the next round
  }
}

// Candidates of event e at offsets[e] .. offsets[e + 1] - 1 (entries >= cap are dropped).
__global__ __launch_bounds__(kCountThreads) void cand_write_kernel(const CandArgs p) {
  __shared__ int wtot[kCountThreads / 64];
  const int e = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const Range r = event_range(p, e);
  const int base = p.offsets[e];
  int running = 0;
  for (int chunk = 0; chunk < r.n; chunk += kCountThreads) {
    const int i = chunk + tid;
    const int row = r.start + i;
    const int c = i < r.n ? p.cls[row] : 0;
    const bool keep = c != 0;
    const unsigned long long m = __ballot(keep);
    const int pre = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wtot[wave] = __popcll(m);
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kCountThreads / 64; ++w) {
      before += w < wave ? wtot[w] : 0;
      all += wtot[w];
    }
    if (keep) {
      const int k = base + running + before + pre;
      if (k < p.cap) {
        p.cand_row[k] = row;
        p.cand_cls[k] = c;
        if (p.cand_kin) *(float4*)(p.cand_kin + 4 * (int64_t)k) = *(const float4*)(p.decoded + 4 * (int64_t)row);
      }
    }
    running += all;
    __syncthreads();  // wtot is rewritten by the next chunk
  }
}

}  // namespace

hipError_t launch_candidates(const CandArgs& p, hipStream_t s) {
  if (p.n_events > 0) {
    hipLaunchKernelGGL(cand_count_kernel, dim3((unsigned)p.n_events), dim3(kCountThreads), 0, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(cand_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || p.n_events == 0) return e;
  hipLaunchKernelGGL(cand_write_kernel, dim3((unsigned)p.n_events), dim3(kCountThreads), 0, s, p);
  return hipGetLastError();
}

}  // namespace mlpf
