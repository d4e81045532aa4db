// Fused position-wise feed-forward block of one encoder layer, BF16 (paper Sec. 5.3):
//   h[M][D] += GELU(y W1 + b1) W2 + b2,   y = LN2(h), h and y in bf16, W1 [D][d_ff], W2 [d_ff][D].
// y is read as given, or computed from h in registers (LN2 fused, bitwise equal to the LayerNorm
// kernel).
// The d_ff-wide intermediate never leaves the workgroup: it is produced and consumed in chunks of
// kFfnHC hidden units. A workgroup owns kFfnBM rows; per chunk
//   phase 1: U^T = W1_c^T y^T (32x32 MFMA blocks; y's fragments stay in registers for the whole
//            workgroup) -> + b1 -> GELU -> bf16, written to LDS as U [row][hidden]; the transposed
//            product puts each lane on one row with the hidden units of that row in its registers,
//            so the LDS writes are 8-byte runs;
//   phase 2: O += U W2_c (U and W2_c^T fragments from LDS).
// The weight chunks are stored pre-tiled in HBM exactly as their LDS images (padded rows, see
// ffn_pack_bytes) and copied linearly with direct-to-LDS loads, double buffered: chunk c+1 travels
// while chunk c is computed. The summation order over k (D in phase 1, d_ff in phase 2) is the order
// of the unfused products, so the results match the two-GEMM path bit for bit. Two shapes: 128 rows
// per workgroup of 8 waves with double-buffered weights, or 64 rows per workgroup of 4 waves with
// single-buffered weights (two workgroups per CU).
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace mlpf {

namespace {

constexpr int kFfnHC = 64;  // hidden units per chunk

// The hidden activation: GELU (the logistic form of the bf16 paths, gelu_fast), or ReLU (the
// paper's network).
template <bool RELU>
__device__ __forceinline__ float hidden_act(float z) {
  if constexpr (RELU) return fmaxf(z, 0.f);
  else return gelu_fast(z);
}

// LDS image of one workgroup: W1 and W2^T chunk buffers (two of each when double buffered), the U
// tile, and (reusing the same bytes after the chunk loop) the FP32 epilogue staging.
template <int D, int BM, bool DBUF>
struct FfnLayout {
  static constexpr int W1RS = 2 * D + 16;       // W1 chunk row: one hidden unit, D k-values
  static constexpr int W1CH = kFfnHC * W1RS;
  static constexpr int W2RS = 2 * kFfnHC + 16;  // W2^T chunk row: one output, kFfnHC k-values
  static constexpr int W2CH = D * W2RS;
  static constexpr int NBUF = DBUF ? 2 : 1;
  static constexpr int URS = 2 * kFfnHC + 16;   // U row: one token row, kFfnHC hidden units
  static constexpr int U_BYTES = BM * URS;
  static constexpr int LN_OFF = NBUF * (W1CH + W2CH) + U_BYTES;  // LN2 gamma, beta (FP32)
  static constexpr int LDS = LN_OFF + 2 * D * 4;
  static constexpr int SRS = 4 * D + 16;        // epilogue staging row (FP32)
  static_assert(BM * SRS <= LDS, "epilogue staging does not fit");
};

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) const void gbl_void;

// Copies `bytes` (a multiple of 16) from global src to LDS dst with NT threads: round r, wave w,
// lane l moves the 16 bytes at offset 16 NT r + 1024 w + 16 l (direct-to-LDS loads write lane l's
// data at the wave's LDS base + 16 l).
template <int NT>
__device__ __forceinline__ void copy_to_lds(const char* src, char* dst, int bytes, int wave, int lane) {
  for (int base = wave * 1024; base < bytes; base += 16 * NT) {
    const int off = base + 16 * lane;
    if (off < bytes)
      __builtin_amdgcn_global_load_lds((gbl_void*)(src + off), (lds_void*)(dst + base), 16, 0, 0);
  }
}

// LayerNorm of the rows held as y fragments (in place): lane (i, h) holds columns 16 g + 8 h + 0..7
// of its row for g < KG, the lane 32 apart the other half. The sums reproduce the LayerNorm
// kernel's exactly: there lane L = 4 g + 2 h + e holds columns 4L .. 4L+3 (e = the two halves of a
// fragment) and a butterfly over lane offsets 32 .. 1 adds partners; offsets above the row's lanes
// add zeros (no change), the next ones pair g with g ^ (KG/2) .. g ^ 1, then h (the lane 32 apart),
// then e. Every lane of the wave must call it (shuffles).
template <int KG>
__device__ __forceinline__ void ln_fragments(u32x4* yf, int h, const float* gam, const float* bet,
                                             float eps) {
  constexpr int D = 16 * KG;
  float t0[KG], t1[KG];
#pragma unroll
  for (int g = 0; g < KG; ++g) {
    float x[8];
    unpack_bf16x8(yf[g], x);
    t0[g] = add_nc(0.f, ln_sum4(x[0], x[1], x[2], x[3]));
    t1[g] = add_nc(0.f, ln_sum4(x[4], x[5], x[6], x[7]));
  }
#pragma unroll
  for (int w = KG / 2; w >= 1; w >>= 1)
#pragma unroll
    for (int g = 0; g < w; ++g) {
      t0[g] = add_nc(t0[g], t0[g + w]);
      t1[g] = add_nc(t1[g], t1[g + w]);
    }
  const float s0 = add_nc(t0[0], __shfl_xor(t0[0], 32, 64));
  const float s1 = add_nc(t1[0], __shfl_xor(t1[0], 32, 64));
  const float mu = ln_mean(add_nc(s0, s1), D);
#pragma unroll
  for (int g = 0; g < KG; ++g) {
    float x[8];
    unpack_bf16x8(yf[g], x);
    t0[g] = add_nc(0.f, ln_sq4(x[0], x[1], x[2], x[3], mu));
    t1[g] = add_nc(0.f, ln_sq4(x[4], x[5], x[6], x[7], mu));
  }
#pragma unroll
  for (int w = KG / 2; w >= 1; w >>= 1)
#pragma unroll
    for (int g = 0; g < w; ++g) {
      t0[g] = add_nc(t0[g], t0[g + w]);
      t1[g] = add_nc(t1[g], t1[g + w]);
    }
  const float q0 = add_nc(t0[0], __shfl_xor(t0[0], 32, 64));
  const float q1 = add_nc(t1[0], __shfl_xor(t1[0], 32, 64));
  const float rs = ln_rstd(add_nc(q0, q1), D, eps);
  // One base address per array (the empty asm keeps the compiler from forming one per fragment):
  // the fragments' offsets 64 g are immediates.
  int hoff = 8 * h;
  __asm__ volatile("" : "+v"(hoff));
  const float* gh = gam + hoff;
  const float* bh = bet + hoff;
#pragma unroll
  for (int g = 0; g < KG; ++g) {
    float x[8];
    unpack_bf16x8(yf[g], x);
    const f32x4 g0 = *(const f32x4*)(gh + 16 * g), g1 = *(const f32x4*)(gh + 16 * g + 4);
    const f32x4 b0 = *(const f32x4*)(bh + 16 * g), b1 = *(const f32x4*)(bh + 16 * g + 4);
    const u32x2 lo = pack_bf16x4(ln_out(x[0], mu, rs, g0[0], b0[0]), ln_out(x[1], mu, rs, g0[1], b0[1]),
                                 ln_out(x[2], mu, rs, g0[2], b0[2]), ln_out(x[3], mu, rs, g0[3], b0[3]));
    const u32x2 hi = pack_bf16x4(ln_out(x[4], mu, rs, g1[0], b1[0]), ln_out(x[5], mu, rs, g1[1], b1[1]),
                                 ln_out(x[6], mu, rs, g1[2], b1[2]), ln_out(x[7], mu, rs, g1[3], b1[3]));
    yf[g] = u32x4{lo[0], lo[1], hi[0], hi[1]};
  }
}

// BM rows per workgroup of NW waves. DBUF: the next chunk's W1 and W2 travel during the current
// chunk (one workgroup per CU at d_model 256). Single buffered: W1 of chunk c+1 is fetched during
// phase 2 of chunk c, W2 after it, and the LDS image is small enough for two workgroups per CU,
// which then hide each other's waits.
template <int D, int BM, int NW, bool DBUF, bool RELU>
__global__ __launch_bounds__(NW * 64) void ffn_fused_kernel(const FfnArgs p) {
  using L = FfnLayout<D, BM, DBUF>;
  constexpr int NT = NW * 64;
  constexpr int KG1 = D / 16;                    // k-groups of phase 1
  constexpr int KG2 = kFfnHC / 16;               // k-groups of phase 2
  constexpr int WN2 = D / 32 < 4 ? D / 32 : 4;   // phase-2 wave grid (rows x columns)
  constexpr int WM2 = NW / WN2;
  constexpr int FM2 = (BM / 32) / WM2, FN2 = (D / 32) / WN2;
  static_assert(FM2 >= 1 && FN2 >= 1 && WM2 * FM2 * 32 == BM && (BM / 32) * (kFfnHC / 32) == NW,
                "bad FFN shape");

  __shared__ __attribute__((aligned(16))) char smem[L::LDS];
  char* const w1buf = smem;                      // [NBUF][W1CH]
  char* const w2buf = smem + L::NBUF * L::W1CH;  // [NBUF][W2CH]
  char* const ubuf = w2buf + L::NBUF * L::W2CH;  // [BM][URS]

  int M = p.M;
  if (p.m_dev) M = min(M, max(*p.m_dev, 0));
  const int m0 = blockIdx.x * BM;
  if (m0 >= M) return;  // uniform over the workgroup

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 31, h = lane >> 5;
  // Hidden chunks c0 .. c1-1: all of them, or part blockIdx.y of p.split equal parts.
  const int per = p.d_ff / kFfnHC / p.split;
  const int c0 = per * (int)blockIdx.y, c1 = c0 + per;
  const char* w1p = (const char*)p.w1p;
  const char* w2p = (const char*)p.w2p;

  copy_to_lds<NT>(w1p + (size_t)c0 * L::W1CH, w1buf, L::W1CH, wave, lane);
  copy_to_lds<NT>(w2p + (size_t)c0 * L::W2CH, w2buf, L::W2CH, wave, lane);

  // Phase-1 role: hidden block hb (32 units of the chunk) x token block tb (32 rows).
  const int hb = wave / (BM / 32), tb = wave % (BM / 32);
  // y fragments (B operand of U^T = W1^T y^T): lane holds row 32 tb + i, k = 16 g + 8 h .. + 7.
  u32x4 yf[KG1];
  {
    const int row = m0 + 32 * tb + i;
    const __bf16* yr = (const __bf16*)p.y + (int64_t)row * D;
#pragma unroll
    for (int g = 0; g < KG1; ++g)
      yf[g] = row < M ? *(const u32x4*)(yr + 16 * g + 8 * h) : u32x4{0, 0, 0, 0};
  }
  if (p.ln_in_g) {
    // gamma and beta through LDS (one copy, short latency) rather than per fragment from memory.
    const float* lg = (const float*)(smem + L::LN_OFF);
    copy_to_lds<NT>((const char*)p.ln_in_g, smem + L::LN_OFF, D * 4, wave, lane);
    copy_to_lds<NT>((const char*)p.ln_in_b, smem + L::LN_OFF + D * 4, D * 4, wave, lane);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    ln_fragments<KG1>(yf, h, lg, lg + D, p.ln_in_eps);
  }
  // Phase-2 role: FM2 x FN2 blocks of 32x32 outputs.
  const int wm2 = wave / WN2, wn2 = wave % WN2;
  f32x16 acc[FM2][FN2];
#pragma unroll
  for (int a = 0; a < FM2; ++a)
#pragma unroll
    for (int b = 0; b < FN2; ++b) acc[a][b] = f32x16{};

  // b1 values of a chunk are loaded one chunk ahead: the wait at the end of each chunk covers them,
  // so GELU never waits on the weight copies in flight (outstanding loads complete in issue order,
  // and the copies' count is not known to the compiler).
  f32x4 bq_next[4];
  auto load_b1 = [&](int c) {
    const float* b1 = p.b1 + c * kFfnHC + 32 * hb + 4 * h;
#pragma unroll
    for (int q = 0; q < 4; ++q) bq_next[q] = *(const f32x4*)(b1 + 8 * q);
  };
  load_b1(c0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  for (int c = c0; c < c1; ++c) {
    const int buf = DBUF ? ((c - c0) & 1) : 0;
    f32x4 bq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) bq[q] = bq_next[q];
    if (c + 1 < c1) load_b1(c + 1);
    if (DBUF && c + 1 < c1) {
      copy_to_lds<NT>(w1p + (size_t)(c + 1) * L::W1CH, w1buf + (buf ^ 1) * L::W1CH, L::W1CH, wave, lane);
      copy_to_lds<NT>(w2p + (size_t)(c + 1) * L::W2CH, w2buf + (buf ^ 1) * L::W2CH, L::W2CH, wave, lane);
    }
    // Phase 1: this wave's 32x32 block of U^T, summed over k = 0 .. D-1 in order.
    {
      const char* w1 = w1buf + buf * L::W1CH + (32 * hb + i) * L::W1RS + 16 * h;
      // The W1 fragments are read in two halves, each issued before its MFMAs (one LDS wait per
      // half rather than one per fragment pair).
      f32x16 u = f32x16{};
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        u32x4 wf[KG1 / 2];
#pragma unroll
        for (int g = 0; g < KG1 / 2; ++g) wf[g] = *(const u32x4*)(w1 + 32 * (half * KG1 / 2 + g));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int g = 0; g < KG1 / 2; ++g) mma_kg<BF16>(wf[g], yf[half * KG1 / 2 + g], u);
      }
      // Lane holds row 32 tb + i and hidden units 32 hb + 8 q + 4 h + (0..3) in registers 4q..4q+3.
      char* urow = ubuf + (32 * tb + i) * L::URS + (32 * hb + 4 * h) * 2;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        *(u32x2*)(urow + 16 * q) =
            pack_bf16x4(hidden_act<RELU>(u[4 * q] + bq[q][0]), hidden_act<RELU>(u[4 * q + 1] + bq[q][1]),
                        hidden_act<RELU>(u[4 * q + 2] + bq[q][2]), hidden_act<RELU>(u[4 * q + 3] + bq[q][3]));
      }
    }
    __syncthreads();
    if (!DBUF && c + 1 < c1)  // W1 is free once every wave is past phase 1
      copy_to_lds<NT>(w1p + (size_t)(c + 1) * L::W1CH, w1buf, L::W1CH, wave, lane);
    // Phase 2: O += U W2_c over the chunk's k-groups in order.
    {
      const char* w2 = w2buf + buf * L::W2CH;
#pragma unroll
      for (int g = 0; g < KG2; ++g) {
        u32x4 af[FM2], bf[FN2];
#pragma unroll
        for (int a = 0; a < FM2; ++a)
          af[a] = *(const u32x4*)(ubuf + (32 * (wm2 * FM2 + a) + i) * L::URS + 32 * g + 16 * h);
#pragma unroll
        for (int b = 0; b < FN2; ++b)
          bf[b] = *(const u32x4*)(w2 + (32 * (wn2 * FN2 + b) + i) * L::W2RS + 32 * g + 16 * h);
#pragma unroll
        for (int a = 0; a < FM2; ++a)
#pragma unroll
          for (int b = 0; b < FN2; ++b) mma_kg<BF16>(af[a], bf[b], acc[a][b]);
      }
    }
    if (!DBUF && c + 1 < c1) {
      __syncthreads();  // W2 is free once every wave is past phase 2
      copy_to_lds<NT>(w2p + (size_t)(c + 1) * L::W2CH, w2buf, L::W2CH, wave, lane);
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copies for chunk c+1 have landed
    __syncthreads();
  }

  // Epilogue: out + b2 staged through LDS as FP32 rows, then h = bf16(h + out) in 16-byte row
  // chunks (8 values; the sum in FP32). Lane l of a 32x32 block holds column l%32 of rows
  // 8*(r/4) + 4*(l/32) + r%4. The h chunks this thread updates are loaded first, so that their
  // latency passes during the staging.
  constexpr int CPR = D / 8;
  constexpr int ROUNDS = BM * CPR / NT;
  static_assert(BM * CPR % NT == 0 && NT % CPR == 0, "epilogue rounds");
  if (p.part) {
    // One part of a split: the FP32 product U W2 over this part's chunks, rows staged through LDS
    // and written as 32-byte runs to part [split][M][D] (no bias, no residual: the reduction
    // kernel adds the parts in order, then b2, then h).
#pragma unroll
    for (int a = 0; a < FM2; ++a)
#pragma unroll
      for (int b = 0; b < FN2; ++b) {
        const int col = 32 * (wn2 * FN2 + b) + i;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 32 * (wm2 * FM2 + a) + 8 * (r >> 2) + 4 * h + (r & 3);
          *(float*)(smem + row * L::SRS + col * 4) = acc[a][b][r];
        }
      }
    __syncthreads();
    float* part = p.part + (int64_t)blockIdx.y * p.M * D;
#pragma unroll
    for (int q = 0; q < ROUNDS; ++q) {
      const int t = tid + q * NT, row = t / CPR, col = (t % CPR) * 8;
      if (m0 + row < M) {
        float* dst = part + (int64_t)(m0 + row) * D + col;
        *(f32x4*)dst = *(const f32x4*)(smem + row * L::SRS + col * 4);
        *(f32x4*)(dst + 4) = *(const f32x4*)(smem + row * L::SRS + col * 4 + 16);
      }
    }
    return;
  }
  // Every round of this thread covers the same 8 columns: their LN gamma and beta load once.
  f32x4 lng[2], lnb[2];
  if (p.y_next) {
    const int col = (tid % CPR) * 8;
    lng[0] = *(const f32x4*)(p.ln_g + col);
    lng[1] = *(const f32x4*)(p.ln_g + col + 4);
    lnb[0] = *(const f32x4*)(p.ln_b + col);
    lnb[1] = *(const f32x4*)(p.ln_b + col + 4);
  }
  u32x4 hv[ROUNDS];
#pragma unroll
  for (int q = 0; q < ROUNDS; ++q) {
    const int t = tid + q * NT, row = t / CPR, col = (t % CPR) * 8;
    hv[q] = m0 + row < M ? *(const u32x4*)((const __bf16*)p.h + (int64_t)(m0 + row) * D + col)
                         : u32x4{0, 0, 0, 0};
  }
#pragma unroll
  for (int a = 0; a < FM2; ++a)
#pragma unroll
    for (int b = 0; b < FN2; ++b) {
      const int col = 32 * (wn2 * FN2 + b) + i;
      const float bias = p.b2[col];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * (wm2 * FM2 + a) + 8 * (r >> 2) + 4 * h + (r & 3);
        *(float*)(smem + row * L::SRS + col * 4) = acc[a][b][r] + bias;
      }
    }
  __syncthreads();
  // CPR consecutive threads own one row (8 values each); they share the row's LayerNorm
  // statistics when the next block's LN1 is fused here (y_next), with the reduction tree of the
  // LayerNorm kernel (its lane l holds values 4l..4l+3: thread j = its lanes 2j, 2j+1), so the
  // output matches that kernel bit for bit.
#pragma unroll
  for (int q = 0; q < ROUNDS; ++q) {
    const int t = tid + q * NT, row = t / CPR, col = (t % CPR) * 8;
    const bool live = m0 + row < M;
    u32x4* dst = (u32x4*)((__bf16*)p.h + (int64_t)(m0 + row) * D + col);
    const u32x4 o = hv[q];
    const f32x4 v0 = *(const f32x4*)(smem + row * L::SRS + col * 4);
    const f32x4 v1 = *(const f32x4*)(smem + row * L::SRS + col * 4 + 16);
    const u32x2 lo = pack_bf16x4(v0[0] + __uint_as_float(o[0] << 16), v0[1] + __uint_as_float(o[0] & 0xffff0000u),
                                 v0[2] + __uint_as_float(o[1] << 16), v0[3] + __uint_as_float(o[1] & 0xffff0000u));
    const u32x2 hi = pack_bf16x4(v1[0] + __uint_as_float(o[2] << 16), v1[1] + __uint_as_float(o[2] & 0xffff0000u),
                                 v1[2] + __uint_as_float(o[3] << 16), v1[3] + __uint_as_float(o[3] & 0xffff0000u));
    const u32x4 hn = u32x4{lo[0], lo[1], hi[0], hi[1]};
    if (live) *dst = hn;
    if (p.y_next) {
      float x[8];
      unpack_bf16x8(hn, x);
      const u32x4 yn = ln_row_chunk8<CPR>(x, lng[0], lng[1], lnb[0], lnb[1], p.ln_eps);
      if (live) *(u32x4*)((__bf16*)p.y_next + (int64_t)(m0 + row) * D + col) = yn;
    }
  }
}

// Reduction of a split FFN: h = bf16(h + ((part_0 + part_1 + ...) + b2)) per row, parts added in
// order in FP32, and the next block's LN1 of the new h when y_next is set (the LayerNorm kernel's
// reduction tree, as in the fused epilogue). CPR = D / 8 consecutive threads own one row, 8 values
// each; all of a thread's loads are issued before the sums.
template <int D, int S>
__global__ __launch_bounds__(256) void ffn_reduce_kernel(const FfnArgs p) {
  constexpr int CPR = D / 8;
  int M = p.M;
  if (p.m_dev) M = min(M, max(*p.m_dev, 0));
  const int t = (int)blockIdx.x * 256 + (int)threadIdx.x;
  const int row = t / CPR, col = (t % CPR) * 8;
  if ((row - row % (256 / CPR)) >= M) return;  // uniform over the workgroup's rows
  const bool live = row < M;
  float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  u32x4 o = u32x4{0, 0, 0, 0};
  if (live) {
    o = *(const u32x4*)((const __bf16*)p.h + (int64_t)row * D + col);
    f32x4 pa[S], pb[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float* src = p.part + ((int64_t)s * p.M + row) * D + col;
      pa[s] = *(const f32x4*)src;
      pb[s] = *(const f32x4*)(src + 4);
    }
    const f32x4 b0 = *(const f32x4*)(p.b2 + col), b1 = *(const f32x4*)(p.b2 + col + 4);
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[e] += pa[s][e];
        v[4 + e] += pb[s][e];
      }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[e] += b0[e];
      v[4 + e] += b1[e];
    }
  }
  const u32x2 lo = pack_bf16x4(v[0] + __uint_as_float(o[0] << 16), v[1] + __uint_as_float(o[0] & 0xffff0000u),
                               v[2] + __uint_as_float(o[1] << 16), v[3] + __uint_as_float(o[1] & 0xffff0000u));
  const u32x2 hi = pack_bf16x4(v[4] + __uint_as_float(o[2] << 16), v[5] + __uint_as_float(o[2] & 0xffff0000u),
                               v[6] + __uint_as_float(o[3] << 16), v[7] + __uint_as_float(o[3] & 0xffff0000u));
  const u32x4 hn = u32x4{lo[0], lo[1], hi[0], hi[1]};
  if (live) *(u32x4*)((__bf16*)p.h + (int64_t)row * D + col) = hn;
  if (p.y_next) {
    float x[8];
    unpack_bf16x8(hn, x);
    const f32x4 g0 = *(const f32x4*)(p.ln_g + col), g1 = *(const f32x4*)(p.ln_g + col + 4);
    const f32x4 e0 = *(const f32x4*)(p.ln_b + col), e1 = *(const f32x4*)(p.ln_b + col + 4);
    const u32x4 yn = ln_row_chunk8<CPR>(x, g0, g1, e0, e1, p.ln_eps);
    if (live) *(u32x4*)((__bf16*)p.y_next + (int64_t)row * D + col) = yn;
  }
}

// Persistent form of the 128-row, 8-wave shape: one workgroup per CU loops over row tiles, so that
// what the one-tile-per-workgroup form pays at the start and end of every tile overlaps work:
// the next tile's first weight chunk (with its b1 values) travels during this tile's last chunk,
// into the buffer that chunk does not use; this tile's residual rows are loaded right after the
// last chunk's products; the stores drain while the next tile computes; LN2's gamma and beta are
// loaded once. The epilogue stages half a tile at a time in the weight buffer the last chunk used.
// Chunk buffers alternate across tiles (par = buffer of a tile's first chunk), so any chunk count
// works. Arithmetic and summation order are those of ffn_fused_kernel (same bits).
template <int D, bool RELU>
__global__ __launch_bounds__(512) void ffn_persistent_kernel(const FfnArgs p) {
  constexpr int BM = 128, NW = 8, NT = NW * 64, HALF = BM / 2;
  constexpr int W1RS = 2 * D + 16, W1CH = kFfnHC * W1RS;
  constexpr int W2RS = 2 * kFfnHC + 16, W2CH = D * W2RS;
  constexpr int B1_OFF = W1CH + W2CH;
  constexpr int BUF = B1_OFF + kFfnHC * 4;  // one chunk: W1 image, W2^T image, b1 values
  constexpr int URS = 2 * kFfnHC + 16;
  constexpr int U_OFF = 2 * BUF;
  constexpr int LN_OFF = U_OFF + BM * URS;
  constexpr int LDS = LN_OFF + 2 * D * 4;
  constexpr int SRS = 4 * D + 16;
  static_assert(HALF * SRS <= BUF, "half-tile staging does not fit a chunk buffer");
  constexpr int KG1 = D / 16, KG2 = kFfnHC / 16;
  constexpr int WN2 = D / 32 < 4 ? D / 32 : 4;
  constexpr int WM2 = NW / WN2;
  constexpr int FM2 = (BM / 32) / WM2, FN2 = (D / 32) / WN2;
  static_assert(FM2 >= 1 && FN2 >= 1 && WM2 * FM2 * 32 == BM && FM2 * 32 <= HALF, "bad FFN shape");
  constexpr int CPR = D / 8;                  // epilogue threads per row (8 values each)
  constexpr int RH = HALF * CPR / NT;         // epilogue rounds per half tile
  static_assert(HALF * CPR % NT == 0 && NT % CPR == 0, "epilogue rounds");

  __shared__ __attribute__((aligned(16))) char smem[LDS];
  char* const ubuf = smem + U_OFF;
  const float* lg = (const float*)(smem + LN_OFF);

  int M = p.M;
  if (p.m_dev) M = min(M, max(*p.m_dev, 0));
  const int ntiles = (M + BM - 1) / BM;
  int tile = blockIdx.x;
  if (tile >= ntiles) return;  // uniform over the workgroup

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 31, h = lane >> 5;
  const int nch = p.d_ff / kFfnHC;
  const char* w1p = (const char*)p.w1p;
  const char* w2p = (const char*)p.w2p;
  const int hb = wave / (BM / 32), tb = wave % (BM / 32);  // phase-1 role
  const int wm2 = wave / WN2, wn2 = wave % WN2;            // phase-2 role
  const int whalf = 32 * wm2 * FM2 / HALF;                 // the half tile holding this wave's rows

  auto copy_chunk = [&](int c, int b) {
    copy_to_lds<NT>(w1p + (size_t)c * W1CH, smem + b * BUF, W1CH, wave, lane);
    copy_to_lds<NT>(w2p + (size_t)c * W2CH, smem + b * BUF + W1CH, W2CH, wave, lane);
    copy_to_lds<NT>((const char*)(p.b1 + c * kFfnHC), smem + b * BUF + B1_OFF, kFfnHC * 4, wave, lane);
  };
  // Rows beyond M read row M-1 instead (no branches around the loads); rows are independent
  // through both products and the LayerNorm, and those rows are never stored.
  u32x4 yf[KG1];
  auto load_y = [&](int m0) {
    const int row = min(m0 + 32 * tb + i, M - 1);
    const __bf16* yr = (const __bf16*)p.y + (int64_t)row * D;
#pragma unroll
    for (int g = 0; g < KG1; ++g) yf[g] = *(const u32x4*)(yr + 16 * g + 8 * h);
  };

  if (p.ln_in_g) {  // LN2 gamma and beta stay in LDS for every tile
    copy_to_lds<NT>((const char*)p.ln_in_g, smem + LN_OFF, D * 4, wave, lane);
    copy_to_lds<NT>((const char*)p.ln_in_b, smem + LN_OFF + D * 4, D * 4, wave, lane);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  copy_chunk(0, 0);
  int par = 0;

  for (;;) {
    const int m0 = tile * BM;
    const int next = tile + (int)gridDim.x;
    const bool has_next = next < ntiles;
    load_y(m0);
    if (p.ln_in_g) ln_fragments<KG1>(yf, h, lg, lg + D, p.ln_in_eps);
    f32x16 acc[FM2][FN2];
#pragma unroll
    for (int a = 0; a < FM2; ++a)
#pragma unroll
      for (int b = 0; b < FN2; ++b) acc[a][b] = f32x16{};
    // The tile's first chunk has landed (and the previous epilogue is done with the staging
    // buffer, which the copies below reuse).
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    for (int c = 0; c < nch; ++c) {
      const int buf = par ^ (c & 1);
      const bool more = c + 1 < nch;
      if (more || has_next) copy_chunk(more ? c + 1 : 0, buf ^ 1);  // next chunk, or next tile's first
      // Phase 1: this wave's 32x32 block of U^T, summed over k = 0 .. D-1 in order.
      {
        const char* w1 = smem + buf * BUF + (32 * hb + i) * W1RS + 16 * h;
        f32x16 u = f32x16{};
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          u32x4 wf[KG1 / 2];
#pragma unroll
          for (int g = 0; g < KG1 / 2; ++g) wf[g] = *(const u32x4*)(w1 + 32 * (half * KG1 / 2 + g));
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int g = 0; g < KG1 / 2; ++g) mma_kg<BF16>(wf[g], yf[half * KG1 / 2 + g], u);
        }
        // Lane holds row 32 tb + i and hidden units 32 hb + 8 q + 4 h + (0..3) in registers 4q..4q+3.
        const float* b1 = (const float*)(smem + buf * BUF + B1_OFF) + 32 * hb + 4 * h;
        f32x4 bq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) bq[q] = *(const f32x4*)(b1 + 8 * q);
        char* urow = ubuf + (32 * tb + i) * URS + (32 * hb + 4 * h) * 2;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          *(u32x2*)(urow + 16 * q) =
              pack_bf16x4(hidden_act<RELU>(u[4 * q] + bq[q][0]), hidden_act<RELU>(u[4 * q + 1] + bq[q][1]),
                          hidden_act<RELU>(u[4 * q + 2] + bq[q][2]), hidden_act<RELU>(u[4 * q + 3] + bq[q][3]));
        }
      }
      __syncthreads();
      // Phase 2: O += U W2_c over the chunk's k-groups in order.
      {
        const char* w2 = smem + buf * BUF + W1CH;
#pragma unroll
        for (int g = 0; g < KG2; ++g) {
          u32x4 af[FM2], bf[FN2];
#pragma unroll
          for (int a = 0; a < FM2; ++a)
            af[a] = *(const u32x4*)(ubuf + (32 * (wm2 * FM2 + a) + i) * URS + 32 * g + 16 * h);
#pragma unroll
          for (int b = 0; b < FN2; ++b)
            bf[b] = *(const u32x4*)(w2 + (32 * (wn2 * FN2 + b) + i) * W2RS + 32 * g + 16 * h);
#pragma unroll
          for (int a = 0; a < FM2; ++a)
#pragma unroll
            for (int b = 0; b < FN2; ++b) mma_kg<BF16>(af[a], bf[b], acc[a][b]);
        }
      }
      if (more) {
        __builtin_amdgcn_s_waitcnt(0);  // this wave's copies for chunk c+1 have landed
        __syncthreads();
      }
    }
    const int bl = par ^ ((nch - 1) & 1);  // buffer of the last chunk: the staging area now

    // Residual rows of this tile. The epilogue's thread index goes through an empty asm statement so that its addresses are formed
    // here rather than hoisted out of the tile loop (where they would stay live across the chunks).
    int etid = tid;
    __asm__ volatile("" : "+v"(etid));
    u32x4 hv[2 * RH];
#pragma unroll
    for (int q = 0; q < 2 * RH; ++q) {
      const int t = etid + q * NT, row = min(m0 + t / CPR, M - 1), col = (t % CPR) * 8;
      hv[q] = *(const u32x4*)((const __bf16*)p.h + (int64_t)row * D + col);
    }
    // The next block's LN1 gamma and beta of the 8 columns this thread updates in every round.
    f32x4 lng[2], lnb[2];
    if (p.y_next) {
      const int col = (etid % CPR) * 8;
      lng[0] = *(const f32x4*)(p.ln_g + col);
      lng[1] = *(const f32x4*)(p.ln_g + col + 4);
      lnb[0] = *(const f32x4*)(p.ln_b + col);
      lnb[1] = *(const f32x4*)(p.ln_b + col + 4);
    }
    __syncthreads();  // every wave is done reading the last chunk's buffer and U

    char* const stage = smem + bl * BUF;
    // This wave's rows within its half tile: row 32 a + 8 (r/4) + (r%4) from srow (constant
    // offsets from one base address).
    int soff = (32 * wm2 * FM2 - HALF * whalf + 4 * h) * SRS + (32 * wn2 * FN2 + i) * 4;
    __asm__ volatile("" : "+v"(soff));
    float bias[FN2];
#pragma unroll
    for (int b = 0; b < FN2; ++b) bias[b] = p.b2[32 * (wn2 * FN2 + b) + i];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if (whalf == half) {
#pragma unroll
        for (int a = 0; a < FM2; ++a)
#pragma unroll
          for (int b = 0; b < FN2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r)
              *(float*)(stage + soff + (32 * a + 8 * (r >> 2) + (r & 3)) * SRS + 128 * b) =
                  acc[a][b][r] + bias[b];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < RH; ++q) {
        const int t = etid + q * NT, row = t / CPR, col = (t % CPR) * 8;
        const int grow = m0 + HALF * half + row;
        const bool live = grow < M;
        const u32x4 o = hv[half * RH + q];
        const f32x4 v0 = *(const f32x4*)(stage + row * SRS + col * 4);
        const f32x4 v1 = *(const f32x4*)(stage + row * SRS + col * 4 + 16);
        const u32x2 lo = pack_bf16x4(v0[0] + __uint_as_float(o[0] << 16), v0[1] + __uint_as_float(o[0] & 0xffff0000u),
                                     v0[2] + __uint_as_float(o[1] << 16), v0[3] + __uint_as_float(o[1] & 0xffff0000u));
        const u32x2 hi = pack_bf16x4(v1[0] + __uint_as_float(o[2] << 16), v1[1] + __uint_as_float(o[2] & 0xffff0000u),
                                     v1[2] + __uint_as_float(o[3] << 16), v1[3] + __uint_as_float(o[3] & 0xffff0000u));
        const u32x4 hn = u32x4{lo[0], lo[1], hi[0], hi[1]};
        if (live) *(u32x4*)((__bf16*)p.h + (int64_t)grow * D + col) = hn;
        if (p.y_next) {
          float x[8];
          unpack_bf16x8(hn, x);
          const u32x4 yn = ln_row_chunk8<CPR>(x, lng[0], lng[1], lnb[0], lnb[1], p.ln_eps);
          if (live) *(u32x4*)((__bf16*)p.y_next + (int64_t)grow * D + col) = yn;
        }
      }
      if (half == 0) __syncthreads();  // the second half reuses the staging rows
    }
    if (!has_next) break;
    tile = next;
    par = bl ^ 1;
  }
}

// Software-pipelined persistent form (chunk counts even): the GELU of chunk c runs while the
// first product of chunk c+1 accumulates, in the same wave, so that the VALU and transcendental
// work of one chunk overlaps the MFMAs of the next instead of following them. W1 therefore
// travels two chunks ahead and W2 (with b1) one chunk ahead: in chunk c, W1 of c+2 goes to buffer
// c%2 and W2, b1 of c+1 to buffer (c+1)%2. The epilogue stages in buffer 1 (the last chunk's);
// the next tile's W1 and W2 of chunk 0 arrive in buffer 0 during the last two chunks, its W1 of
// chunk 1 at the tile's start. Arithmetic and summation order are those of ffn_fused_kernel.
template <int D, bool RELU>
__global__ __launch_bounds__(512) void ffn_pipelined_kernel(const FfnArgs p) {
  constexpr int BM = 128, NW = 8, NT = NW * 64, HALF = BM / 2;
  constexpr int W1RS = 2 * D + 16, W1CH = kFfnHC * W1RS;
  constexpr int W2RS = 2 * kFfnHC + 16, W2CH = D * W2RS;
  constexpr int B1_OFF = W1CH + W2CH;
  constexpr int BUF = B1_OFF + kFfnHC * 4;
  constexpr int URS = 2 * kFfnHC + 16;
  constexpr int U_OFF = 2 * BUF;
  constexpr int LN_OFF = U_OFF + BM * URS;
  constexpr int LDS = LN_OFF + 2 * D * 4;
  constexpr int SRS = 4 * D + 16;
  static_assert(HALF * SRS <= BUF, "half-tile staging does not fit a chunk buffer");
  constexpr int KG1 = D / 16, KG2 = kFfnHC / 16;
  constexpr int WN2 = D / 32 < 4 ? D / 32 : 4;
  constexpr int WM2 = NW / WN2;
  constexpr int FM2 = (BM / 32) / WM2, FN2 = (D / 32) / WN2;
  static_assert(FM2 >= 1 && FN2 >= 1 && WM2 * FM2 * 32 == BM && FM2 * 32 <= HALF, "bad FFN shape");
  static_assert(KG1 % 4 == 0, "first product in four parts");
  constexpr int CPR = D / 8;
  constexpr int RH = HALF * CPR / NT;
  static_assert(HALF * CPR % NT == 0 && NT % CPR == 0, "epilogue rounds");

  __shared__ __attribute__((aligned(16))) char smem[LDS];
  char* const ubuf = smem + U_OFF;
  const float* lg = (const float*)(smem + LN_OFF);

  int M = p.M;
  if (p.m_dev) M = min(M, max(*p.m_dev, 0));
  const int ntiles = (M + BM - 1) / BM;
  int tile = blockIdx.x;
  const int nch = p.d_ff / kFfnHC;
  if (tile >= ntiles || (nch & 1)) return;  // uniform over the workgroup

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 31, h = lane >> 5;
  const char* w1p = (const char*)p.w1p;
  const char* w2p = (const char*)p.w2p;
  const int hb = wave / (BM / 32), tb = wave % (BM / 32);
  const int wm2 = wave / WN2, wn2 = wave % WN2;
  const int whalf = 32 * wm2 * FM2 / HALF;

  // The copies are issued by waves 0-3 only: the waves of the second hidden block (4-7, the
  // younger wave on each SIMD) finish the first product later, and the first four would otherwise
  // wait for them at the barrier after it.
  const bool copier = wave < NW / 2;
  auto copy_w1 = [&](int c, int b) {
    if (copier) copy_to_lds<NT / 2>(w1p + (size_t)c * W1CH, smem + b * BUF, W1CH, wave, lane);
  };
  auto copy_w2 = [&](int c, int b) {
    if (copier) {
      copy_to_lds<NT / 2>(w2p + (size_t)c * W2CH, smem + b * BUF + W1CH, W2CH, wave, lane);
      copy_to_lds<NT / 2>((const char*)(p.b1 + c * kFfnHC), smem + b * BUF + B1_OFF, kFfnHC * 4, wave,
                          lane);
    }
  };
  u32x4 yf[KG1];
  auto load_y = [&](int m0) {
    const int row = min(m0 + 32 * tb + i, M - 1);
    const __bf16* yr = (const __bf16*)p.y + (int64_t)row * D;
#pragma unroll
    for (int g = 0; g < KG1; ++g) yf[g] = *(const u32x4*)(yr + 16 * g + 8 * h);
  };
  // Values 4q..4q+3 of this wave's U^T block (row 32 tb + i, hidden units 32 hb + 8q + 4h + 0..3):
  // + b1, GELU, bf16, to U.
  char* const urow = ubuf + (32 * tb + i) * URS + (32 * hb + 4 * h) * 2;
  auto gelu_part = [&](const f32x16& u, int q, const float* b1s) {
    const f32x4 bq = *(const f32x4*)(b1s + 8 * q);
    *(u32x2*)(urow + 16 * q) =
        pack_bf16x4(hidden_act<RELU>(u[4 * q] + bq[0]), hidden_act<RELU>(u[4 * q + 1] + bq[1]),
                    hidden_act<RELU>(u[4 * q + 2] + bq[2]), hidden_act<RELU>(u[4 * q + 3] + bq[3]));
  };

  if (p.ln_in_g) {
    copy_to_lds<NT>((const char*)p.ln_in_g, smem + LN_OFF, D * 4, wave, lane);
    copy_to_lds<NT>((const char*)p.ln_in_b, smem + LN_OFF + D * 4, D * 4, wave, lane);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  copy_w1(0, 0);
  copy_w2(0, 0);

  for (;;) {
    const int m0 = tile * BM;
    const int next = tile + (int)gridDim.x;
    const bool has_next = next < ntiles;
    copy_w1(1, 1);  // buffer 1 is free: the previous epilogue is done with it
    load_y(m0);
    if (p.ln_in_g) ln_fragments<KG1>(yf, h, lg, lg + D, p.ln_in_eps);
    f32x16 acc[FM2][FN2];
#pragma unroll
    for (int a = 0; a < FM2; ++a)
#pragma unroll
      for (int b = 0; b < FN2; ++b) acc[a][b] = f32x16{};
    __builtin_amdgcn_s_waitcnt(0);  // chunk 0 and W1 of chunk 1 have landed
    __syncthreads();
    // First product of chunk 0 on its own.
    f32x16 u = f32x16{};
    {
      const char* w1 = smem + (32 * hb + i) * W1RS + 16 * h;
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        u32x4 wf[KG1 / 2];
#pragma unroll
        for (int g = 0; g < KG1 / 2; ++g) wf[g] = *(const u32x4*)(w1 + 32 * (half * KG1 / 2 + g));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int g = 0; g < KG1 / 2; ++g) mma_kg<BF16>(wf[g], yf[half * KG1 / 2 + g], u);
      }
    }

    for (int c = 0; c < nch; ++c) {
      const int b = c & 1;
      if (c + 2 < nch) copy_w1(c + 2, b);
      else if (c + 2 == nch && has_next) copy_w1(0, b);
      if (c + 1 < nch) copy_w2(c + 1, b ^ 1);
      else if (has_next) copy_w2(0, b ^ 1);
      const float* b1s = (const float*)(smem + b * BUF + B1_OFF) + 32 * hb + 4 * h;
      f32x16 un = f32x16{};
      if (c + 1 < nch) {
        // GELU of chunk c in four parts, each beside a quarter of chunk c+1's first product.
        const char* w1 = smem + (b ^ 1) * BUF + (32 * hb + i) * W1RS + 16 * h;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          u32x4 wf[KG1 / 4];
#pragma unroll
          for (int g = 0; g < KG1 / 4; ++g) wf[g] = *(const u32x4*)(w1 + 32 * (q * KG1 / 4 + g));
          gelu_part(u, q, b1s);
#pragma unroll
          for (int g = 0; g < KG1 / 4; ++g) mma_kg<BF16>(wf[g], yf[q * KG1 / 4 + g], un);
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) gelu_part(u, q, b1s);
      }
      __syncthreads();
      {
        const char* w2 = smem + b * BUF + W1CH;
#pragma unroll
        for (int g = 0; g < KG2; ++g) {
          u32x4 af[FM2], bf[FN2];
#pragma unroll
          for (int a = 0; a < FM2; ++a)
            af[a] = *(const u32x4*)(ubuf + (32 * (wm2 * FM2 + a) + i) * URS + 32 * g + 16 * h);
#pragma unroll
          for (int bb = 0; bb < FN2; ++bb)
            bf[bb] = *(const u32x4*)(w2 + (32 * (wn2 * FN2 + bb) + i) * W2RS + 32 * g + 16 * h);
#pragma unroll
          for (int a = 0; a < FM2; ++a)
#pragma unroll
            for (int bb = 0; bb < FN2; ++bb) mma_kg<BF16>(af[a], bf[bb], acc[a][bb]);
        }
      }
      if (c + 1 < nch) {
        __builtin_amdgcn_s_waitcnt(0);  // W1 of c+2, W2 and b1 of c+1 have landed
        __syncthreads();                // and U is free again
        u = un;
      }
    }

    int etid = tid;
    __asm__ volatile("" : "+v"(etid));
    u32x4 hv[2 * RH];
#pragma unroll
    for (int q = 0; q < 2 * RH; ++q) {
      const int t = etid + q * NT, row = min(m0 + t / CPR, M - 1), col = (t % CPR) * 8;
      hv[q] = *(const u32x4*)((const __bf16*)p.h + (int64_t)row * D + col);
    }
    f32x4 lng[2], lnb[2];
    if (p.y_next) {
      const int col = (etid % CPR) * 8;
      lng[0] = *(const f32x4*)(p.ln_g + col);
      lng[1] = *(const f32x4*)(p.ln_g + col + 4);
      lnb[0] = *(const f32x4*)(p.ln_b + col);
      lnb[1] = *(const f32x4*)(p.ln_b + col + 4);
    }
    __syncthreads();  // every wave is done reading buffer 1 and U

    char* const stage = smem + BUF;
    int soff = (32 * wm2 * FM2 - HALF * whalf + 4 * h) * SRS + (32 * wn2 * FN2 + i) * 4;
    __asm__ volatile("" : "+v"(soff));
    float bias[FN2];
#pragma unroll
    for (int bb = 0; bb < FN2; ++bb) bias[bb] = p.b2[32 * (wn2 * FN2 + bb) + i];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if (whalf == half) {
#pragma unroll
        for (int a = 0; a < FM2; ++a)
#pragma unroll
          for (int bb = 0; bb < FN2; ++bb)
#pragma unroll
            for (int r = 0; r < 16; ++r)
              *(float*)(stage + soff + (32 * a + 8 * (r >> 2) + (r & 3)) * SRS + 128 * bb) =
                  acc[a][bb][r] + bias[bb];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < RH; ++q) {
        const int t = etid + q * NT, row = t / CPR, col = (t % CPR) * 8;
        const int grow = m0 + HALF * half + row;
        const bool live = grow < M;
        const u32x4 o = hv[half * RH + q];
        const f32x4 v0 = *(const f32x4*)(stage + row * SRS + col * 4);
        const f32x4 v1 = *(const f32x4*)(stage + row * SRS + col * 4 + 16);
        const u32x2 lo = pack_bf16x4(v0[0] + __uint_as_float(o[0] << 16), v0[1] + __uint_as_float(o[0] & 0xffff0000u),
                                     v0[2] + __uint_as_float(o[1] << 16), v0[3] + __uint_as_float(o[1] & 0xffff0000u));
        const u32x2 hi = pack_bf16x4(v1[0] + __uint_as_float(o[2] << 16), v1[1] + __uint_as_float(o[2] & 0xffff0000u),
                                     v1[2] + __uint_as_float(o[3] << 16), v1[3] + __uint_as_float(o[3] & 0xffff0000u));
        const u32x4 hn = u32x4{lo[0], lo[1], hi[0], hi[1]};
        if (live) *(u32x4*)((__bf16*)p.h + (int64_t)grow * D + col) = hn;
        if (p.y_next) {
          float x[8];
          unpack_bf16x8(hn, x);
          const u32x4 yn = ln_row_chunk8<CPR>(x, lng[0], lng[1], lnb[0], lnb[1], p.ln_eps);
          if (live) *(u32x4*)((__bf16*)p.y_next + (int64_t)grow * D + col) = yn;
        }
      }
      __syncthreads();  // the staging rows (buffer 1) are reused next
    }
    if (!has_next) break;
    tile = next;
  }
}

template <int D, bool RELU>
hipError_t launch_pipelined(const FfnArgs& p, hipStream_t s) {
  if ((p.d_ff / kFfnHC) & 1) return hipErrorInvalidValue;
  const int64_t tiles = ((int64_t)p.M + 127) / 128;
  if (tiles == 0) return hipSuccess;
  static int slots[64] = {0};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (slots[dev] == 0) {
    int cus = 0, per_cu = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ffn_pipelined_kernel<D, RELU>, 512, 0);
    if (e != hipSuccess) return e;
    slots[dev] = (cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
  }
  const unsigned grid = (unsigned)(tiles < slots[dev] ? tiles : slots[dev]);
  hipLaunchKernelGGL((ffn_pipelined_kernel<D, RELU>), dim3(grid), dim3(512), 0, s, p);
  return hipGetLastError();
}

template <int D, bool RELU>
hipError_t launch_persistent(const FfnArgs& p, hipStream_t s) {
  const int64_t tiles = ((int64_t)p.M + 127) / 128;
  if (tiles == 0) return hipSuccess;
  // As many workgroups as fit on the device at once (one per CU at d_model 256, where the LDS
  // image takes the CU's whole LDS).
  static int slots[64] = {0};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (slots[dev] == 0) {
    int cus = 0, per_cu = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ffn_persistent_kernel<D, RELU>, 512, 0);
    if (e != hipSuccess) return e;
    slots[dev] = (cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
  }
  const unsigned grid = (unsigned)(tiles < slots[dev] ? tiles : slots[dev]);
  hipLaunchKernelGGL((ffn_persistent_kernel<D, RELU>), dim3(grid), dim3(512), 0, s, p);
  return hipGetLastError();
}

template <int BM, int NW, bool DBUF, bool RELU>
hipError_t launch_v(const FfnArgs& p, hipStream_t s) {
  const int64_t grid = ((int64_t)p.M + BM - 1) / BM;
  if (grid == 0) return hipSuccess;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  const int nch = p.d_ff / kFfnHC;
  if (p.split < 1 || nch % p.split != 0 || (p.split > 1) != (p.part != nullptr)) return hipErrorInvalidValue;
  const dim3 g((unsigned)grid, (unsigned)p.split);
  switch (p.d_model) {
    case 64: hipLaunchKernelGGL((ffn_fused_kernel<64, BM, NW, DBUF, RELU>), g, dim3(NW * 64), 0, s, p); break;
    case 128: hipLaunchKernelGGL((ffn_fused_kernel<128, BM, NW, DBUF, RELU>), g, dim3(NW * 64), 0, s, p); break;
    default: hipLaunchKernelGGL((ffn_fused_kernel<256, BM, NW, DBUF, RELU>), g, dim3(NW * 64), 0, s, p); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || p.split == 1) return e;
  const int64_t rgrid = ((int64_t)p.M * (p.d_model / 8) + 255) / 256;
  auto reduce = [&](auto d_tag) {
    constexpr int DM = decltype(d_tag)::value;
    switch (p.split) {
      case 2: hipLaunchKernelGGL((ffn_reduce_kernel<DM, 2>), dim3((unsigned)rgrid), dim3(256), 0, s, p); break;
      case 4: hipLaunchKernelGGL((ffn_reduce_kernel<DM, 4>), dim3((unsigned)rgrid), dim3(256), 0, s, p); break;
      case 8: hipLaunchKernelGGL((ffn_reduce_kernel<DM, 8>), dim3((unsigned)rgrid), dim3(256), 0, s, p); break;
      default: hipLaunchKernelGGL((ffn_reduce_kernel<DM, 16>), dim3((unsigned)rgrid), dim3(256), 0, s, p); break;
    }
  };
  if (p.split != 2 && p.split != 4 && p.split != 8 && p.split != 16) return hipErrorInvalidValue;
  switch (p.d_model) {
    case 64: reduce(std::integral_constant<int, 64>{}); break;
    case 128: reduce(std::integral_constant<int, 128>{}); break;
    default: reduce(std::integral_constant<int, 256>{}); break;
  }
  return hipGetLastError();
}

}  // namespace

int ffn_fused_supported(int d_model, int d_ff) {
  return (d_model == 64 || d_model == 128 || d_model == 256) && d_ff % kFfnHC == 0 && d_ff > 0;
}

size_t ffn_pack_bytes(int d_model, int d_ff, int which) {
  const size_t chunks = (size_t)d_ff / kFfnHC;
  return which == 1 ? chunks * kFfnHC * (2 * (size_t)d_model + 16)
                    : chunks * (size_t)d_model * (2 * kFfnHC + 16);
}

void ffn_pack(const uint16_t* w1t, const uint16_t* w2t, int d_model, int d_ff, uint16_t* w1p,
              uint16_t* w2p) {
  const int D = d_model, HC = kFfnHC;
  const size_t w1rs = (2 * (size_t)D + 16) / 2, w2rs = (2 * (size_t)HC + 16) / 2;  // in bf16 units
  for (int c = 0; c < d_ff / HC; ++c) {
    uint16_t* b1 = w1p + (size_t)c * HC * w1rs;
    for (int r = 0; r < HC; ++r)
      for (int k = 0; k < w1rs; ++k) b1[r * w1rs + k] = k < D ? w1t[(size_t)(c * HC + r) * D + k] : 0;
    uint16_t* b2 = w2p + (size_t)c * D * w2rs;
    for (int o = 0; o < D; ++o)
      for (int k = 0; k < w2rs; ++k) b2[o * w2rs + k] = k < HC ? w2t[(size_t)o * d_ff + c * HC + k] : 0;
  }
}

// Variants 1 and 2 as declared; 3 = variant 1 as a persistent kernel (ffn_persistent_kernel);
// 4 = the software-pipelined persistent kernel (even chunk counts); 5 and 6 = variants 2 and 1
// over p.split parts of the hidden units (p.part set) plus the reduction kernel.
namespace {
template <bool RELU>
hipError_t launch_variant(const FfnArgs& p, int variant, hipStream_t s) {
  if (variant != 5 && variant != 6 && (p.split != 1 || p.part)) return hipErrorInvalidValue;
  if (variant == 1 || variant == 6) return launch_v<128, 8, true, RELU>(p, s);
  if (variant == 2 || variant == 5) return launch_v<64, 4, false, RELU>(p, s);
  if (variant == 3) {
    switch (p.d_model) {
      case 64: return launch_persistent<64, RELU>(p, s);
      case 128: return launch_persistent<128, RELU>(p, s);
      default: return launch_persistent<256, RELU>(p, s);
    }
  }
  if (variant == 4) {
    switch (p.d_model) {
      case 64: return launch_pipelined<64, RELU>(p, s);
      case 128: return launch_pipelined<128, RELU>(p, s);
      default: return launch_pipelined<256, RELU>(p, s);
    }
  }
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_ffn_fused(const FfnArgs& p, int variant, hipStream_t s) {
  if (!ffn_fused_supported(p.d_model, p.d_ff)) return hipErrorInvalidValue;
  return p.relu ? launch_variant<true>(p, variant, s) : launch_variant<false>(p, variant, s);
}

}  // namespace mlpf
