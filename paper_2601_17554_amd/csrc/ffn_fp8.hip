// Fused position-wise feed-forward block with FP8-E4M3 operands (paper Sec. 5.3 FFN; E4M3 per-tensor
// scaled products with FP32 accumulation):
//   y = E4M3(LN2(h) / s_a1)                         LN2 in registers, FP32 statistics
//   U = E4M3(act(s_a1 s_w1 (y W1) + b1) / s_a2)      chunks of 64 hidden units, never in HBM
//   h = bf16(h + s_a2 s_w2 (U W2) + b2)              residual update in FP32, rounded once
// with W1, W2 E4M3 images. Every product runs on gfx950's 32x32x64 F8F6F4 MFMA (64-value k-groups,
// in k order), the quantisation points and roundings are those of the two-product FP8 path (the
// LayerNorm kernel's E4M3 output, then the GEMM epilogues), so the results are its bits.
//
// One workgroup of 8 waves per CU loops over tiles of 128 rows (persistent). Per chunk of 64 hidden
// units: phase 1, U^T = W1_c^T y^T (each wave one 32x32 block: 4 MFMAs at d_model 256; y's
// fragments stay in registers for the tile), + b1, activation, E4M3, written to LDS as 4-byte
// runs of a row; phase 2, O += U W2_c (each wave 2 x 2 blocks, one MFMA each). The weight chunks,
// stored pre-tiled as their LDS images (ffn_fp8_pack), arrive by direct-to-LDS loads, double
// buffered; the next tile's first chunk travels during the current tile's last. The epilogue
// stages half a tile of FP32 outputs in a region of its own and updates h in 16-byte row chunks,
// optionally writing the next block's LN1 (bf16, the LayerNorm kernel's bits).
#include "common.h"
#include "kernels.h"

namespace mlpf {

namespace {

constexpr int kHC = 64;  // hidden units per chunk (one 64-value k-group of the second product)

template <bool RELU>
__device__ __forceinline__ float act8(float z) {
  if constexpr (RELU) return fmaxf(z, 0.f);
  else return gelu_fast(z);
}

typedef __attribute__((address_space(3))) void lds_void8;
typedef __attribute__((address_space(1))) const void gbl_void8;

template <int NT>
__device__ __forceinline__ void copy_lds8(const char* src, char* dst, int bytes, int wave, int lane) {
  for (int base = wave * 1024; base < bytes; base += 16 * NT) {
    const int off = base + 16 * lane;
    if (off < bytes)
      __builtin_amdgcn_global_load_lds((gbl_void8*)(src + off), (lds_void8*)(dst + base), 16, 0, 0);
  }
}

// The fragments of one row for the first product: lane (i, h) holds bf16 columns 64 g + 32 h + 0..31
// of its row in xf[4 g .. 4 g + 3] (KG = D / 64 groups). LayerNorm of those rows in place, then
// E4M3 of out * scale into yq[2 g], yq[2 g + 1]. The sums reproduce the LayerNorm kernel's tree:
// there lane L = 16 g + 8 h + j holds columns 4L .. 4L+3 and a butterfly over lane offsets
// 32 .. 1 adds partners (offsets beyond the row's lanes add zeros); here the offsets above 8 pair
// groups g in registers, 8 pairs the two lane halves, and 4, 2, 1 pair the j of one lane.
template <int KG>
__device__ __forceinline__ void ln_to_fp8(const u32x4* xf, u32x4* yq, const float* gam,
                                          const float* bet, float eps, float scale, int h) {
  constexpr int D = 64 * KG;
  float t[KG][8];
  auto vals = [&](int g, int j, float* x) {  // the 4 columns of LN-lane (g, h, j)
    const u32x4 w = xf[4 * g + j / 2];
    const int e = (j & 1) * 2;
    x[0] = __uint_as_float(w[e] << 16);
    x[1] = __uint_as_float(w[e] & 0xffff0000u);
    x[2] = __uint_as_float(w[e + 1] << 16);
    x[3] = __uint_as_float(w[e + 1] & 0xffff0000u);
  };
  auto tree = [&]() {
#pragma unroll
    for (int w = KG / 2; w >= 1; w >>= 1)
#pragma unroll
      for (int g = 0; g < w; ++g)
#pragma unroll
        for (int j = 0; j < 8; ++j) t[g][j] = add_nc(t[g][j], t[g + w][j]);
#pragma unroll
    for (int j = 0; j < 8; ++j) t[0][j] = add_nc(t[0][j], __shfl_xor(t[0][j], 32, 64));
#pragma unroll
    for (int w = 4; w >= 1; w >>= 1)
#pragma unroll
      for (int j = 0; j < w; ++j) t[0][j] = add_nc(t[0][j], t[0][j + w]);
    return t[0][0];
  };
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      float x[4];
      vals(g, j, x);
      t[g][j] = add_nc(0.f, ln_sum4(x[0], x[1], x[2], x[3]));
    }
  const float mu = ln_mean(tree(), D);
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      float x[4];
      vals(g, j, x);
      t[g][j] = add_nc(0.f, ln_sq4(x[0], x[1], x[2], x[3], mu));
    }
  const float rs = ln_rstd(tree(), D, eps);
  // One base address per array (the empty asm keeps the compiler from forming, and keeping live
  // across the tile loop, one address per fragment): the offsets 64 g + 4 j are immediates.
  int hoff = 32 * h;
  __asm__ volatile("" : "+v"(hoff));
  const float* gh = gam + hoff;
  const float* bh = bet + hoff;
#pragma unroll
  for (int g = 0; g < KG; ++g) {
    uint32_t q[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      float x[4];
      vals(g, j, x);
      const int col = 64 * g + 4 * j;
      const f32x4 gg = *(const f32x4*)(gh + col), bb = *(const f32x4*)(bh + col);
      q[j] = pack_fp8x4(ln_out(x[0], mu, rs, gg[0], bb[0]) * scale, ln_out(x[1], mu, rs, gg[1], bb[1]) * scale,
                        ln_out(x[2], mu, rs, gg[2], bb[2]) * scale, ln_out(x[3], mu, rs, gg[3], bb[3]) * scale);
    }
    yq[2 * g] = u32x4{q[0], q[1], q[2], q[3]};
    yq[2 * g + 1] = u32x4{q[4], q[5], q[6], q[7]};
  }
}

template <int D, bool RELU>
__global__ __launch_bounds__(512) void ffn_fp8_kernel(const FfnArgs p) {
  constexpr int BM = 128, NW = 8, NT = NW * 64, HALF = BM / 2, KG = D / 64;
  constexpr int W1RS = D + 16, W1CH = kHC * W1RS;      // W1 chunk row: one hidden unit, D bytes
  constexpr int W2RS = kHC + 16, W2CH = D * W2RS;      // W2^T chunk row: one output, 64 bytes
  constexpr int B1_OFF = W1CH + W2CH;
  constexpr int BUF = B1_OFF + kHC * 4;                // one chunk: W1, W2^T images, b1 values
  constexpr int URS = kHC + 16;                        // U row: 64 E4M3 hidden values
  constexpr int U_OFF = 2 * BUF;
  constexpr int LN_OFF = U_OFF + BM * URS;
  constexpr int SRS = 4 * D + 16;                      // epilogue staging row (FP32)
  constexpr int ST_OFF = LN_OFF + 2 * D * 4;
  constexpr int LDS = ST_OFF + HALF * SRS;
  static_assert(LDS <= 160 * 1024, "LDS image too large");
  constexpr int WN2 = D / 32 < 4 ? D / 32 : 4;
  constexpr int WM2 = NW / WN2;
  constexpr int FM2 = (BM / 32) / WM2, FN2 = (D / 32) / WN2;
  static_assert(FM2 >= 1 && FN2 >= 1 && WM2 * FM2 * 32 == BM && FM2 * 32 <= HALF, "bad FFN shape");
  constexpr int CPR = D / 8;
  constexpr int RH = HALF * CPR / NT;
  static_assert(HALF * CPR % NT == 0 && NT % CPR == 0, "epilogue rounds");

  __shared__ __attribute__((aligned(16))) char smem[LDS];
  char* const ubuf = smem + U_OFF;
  char* const stage = smem + ST_OFF;
  const float* lg = (const float*)(smem + LN_OFF);

  int M = p.M;
  if (p.m_dev) M = min(M, max(*p.m_dev, 0));
  const int ntiles = (M + BM - 1) / BM;
  int tile = blockIdx.x;
  if (tile >= ntiles) return;  // uniform over the workgroup

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 31, h = lane >> 5;
  const int nch = p.d_ff / kHC;
  const char* w1p = (const char*)p.w1p;
  const char* w2p = (const char*)p.w2p;
  const int hb = wave / (BM / 32), tb = wave % (BM / 32);  // phase-1 role
  const int wm2 = wave / WN2, wn2 = wave % WN2;            // phase-2 role
  const int whalf = 32 * wm2 * FM2 / HALF;

  auto copy_chunk = [&](int c, int b) {
    copy_lds8<NT>(w1p + (size_t)c * W1CH, smem + b * BUF, W1CH, wave, lane);
    copy_lds8<NT>(w2p + (size_t)c * W2CH, smem + b * BUF + W1CH, W2CH, wave, lane);
    copy_lds8<NT>((const char*)(p.b1 + c * kHC), smem + b * BUF + B1_OFF, kHC * 4, wave, lane);
  };
  // LN2's gamma and beta stay in LDS for every tile.
  copy_lds8<NT>((const char*)p.ln_in_g, smem + LN_OFF, D * 4, wave, lane);
  copy_lds8<NT>((const char*)p.ln_in_b, smem + LN_OFF + D * 4, D * 4, wave, lane);
  copy_chunk(0, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int par = 0;

  for (;;) {
    const int m0 = tile * BM;
    const int next = tile + (int)gridDim.x;
    const bool has_next = next < ntiles;
    // Rows beyond M read row M-1 (rows are independent; those rows are never stored).
    u32x4 yq[2 * KG];
    {
      const int row = min(m0 + 32 * tb + i, M - 1);
      const char* hr = (const char*)p.y + (int64_t)row * D * 2;
      u32x4 xf[4 * KG];
#pragma unroll
      for (int g = 0; g < KG; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) xf[4 * g + e] = *(const u32x4*)(hr + (64 * g + 32 * h) * 2 + 16 * e);
      ln_to_fp8<KG>(xf, yq, lg, lg + D, p.ln_in_eps, p.fp8_in_scale, h);
    }
    f32x16 acc[FM2][FN2];
#pragma unroll
    for (int a = 0; a < FM2; ++a)
#pragma unroll
      for (int b = 0; b < FN2; ++b) acc[a][b] = f32x16{};

    for (int c = 0; c < nch; ++c) {
      const int buf = par ^ (c & 1);
      const bool more = c + 1 < nch;
      if (more || has_next) copy_chunk(more ? c + 1 : 0, buf ^ 1);  // next chunk, or next tile's first
      // Phase 1: this wave's 32x32 block of U^T over k = 0 .. D-1 in 64-value groups.
      {
        const char* w1 = smem + buf * BUF + (32 * hb + i) * W1RS + 32 * h;
        f32x16 u = f32x16{};
        u32x4 wf[2 * KG];
#pragma unroll
        for (int g = 0; g < KG; ++g) {
          wf[2 * g] = *(const u32x4*)(w1 + 64 * g);
          wf[2 * g + 1] = *(const u32x4*)(w1 + 64 * g + 16);
        }
#pragma unroll
        for (int g = 0; g < KG; ++g) mma_fp8_k64(wf[2 * g], wf[2 * g + 1], yq[2 * g], yq[2 * g + 1], u);
        // Lane holds row 32 tb + i and hidden units 32 hb + 8 q + 4 h + (0..3) in registers 4q..4q+3.
        const float* b1 = (const float*)(smem + buf * BUF + B1_OFF) + 32 * hb + 4 * h;
        char* urow = ubuf + (32 * tb + i) * URS + 32 * hb + 4 * h;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const f32x4 bq = *(const f32x4*)(b1 + 8 * q);
          float v[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = act8<RELU>(u[4 * q + e] * p.acc_scale + bq[e]);
          *(uint32_t*)(urow + 8 * q) = pack_fp8x4(v[0] * p.out_scale, v[1] * p.out_scale,
                                                  v[2] * p.out_scale, v[3] * p.out_scale);
        }
      }
      __syncthreads();
      // Phase 2: O += U W2_c, one 64-value k-group.
      {
        const char* w2 = smem + buf * BUF + W1CH;
        u32x4 af[FM2][2], bf[FN2][2];
#pragma unroll
        for (int a = 0; a < FM2; ++a)
#pragma unroll
          for (int e = 0; e < 2; ++e)
            af[a][e] = *(const u32x4*)(ubuf + (32 * (wm2 * FM2 + a) + i) * URS + 32 * h + 16 * e);
#pragma unroll
        for (int b = 0; b < FN2; ++b)
#pragma unroll
          for (int e = 0; e < 2; ++e)
            bf[b][e] = *(const u32x4*)(w2 + (32 * (wn2 * FN2 + b) + i) * W2RS + 32 * h + 16 * e);
#pragma unroll
        for (int a = 0; a < FM2; ++a)
#pragma unroll
          for (int b = 0; b < FN2; ++b) mma_fp8_k64(af[a][0], af[a][1], bf[b][0], bf[b][1], acc[a][b]);
      }
      if (more) {
        __builtin_amdgcn_s_waitcnt(0);  // this wave's copies for chunk c+1 have landed
        __syncthreads();
      }
    }
    const int bl = par ^ ((nch - 1) & 1);  // buffer of the last chunk

    // Residual rows of this tile, and the next block's LN1 gamma and beta of this thread's columns.
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
                  acc[a][b][r] * p.acc_scale2 + bias[b];
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
      __syncthreads();  // the staging rows are reused (second half, next tile)
    }
    if (!has_next) break;
    tile = next;
    par = bl ^ 1;
    // The next tile's first chunk (issued during the last chunk) has landed.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
}

template <int D, bool RELU>
hipError_t launch_fp8_d(const FfnArgs& p, hipStream_t s) {
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
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ffn_fp8_kernel<D, RELU>, 512, 0);
    if (e != hipSuccess) return e;
    slots[dev] = (cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
  }
  const unsigned grid = (unsigned)(tiles < slots[dev] ? tiles : slots[dev]);
  hipLaunchKernelGGL((ffn_fp8_kernel<D, RELU>), dim3(grid), dim3(512), 0, s, p);
  return hipGetLastError();
}

}  // namespace

size_t ffn_fp8_pack_bytes(int d_model, int d_ff, int which) {
  const size_t chunks = (size_t)d_ff / kHC;
  return which == 1 ? chunks * kHC * ((size_t)d_model + 16) : chunks * (size_t)d_model * (kHC + 16);
}

void ffn_fp8_pack(const uint8_t* w1t, const uint8_t* w2t, int d_model, int d_ff, uint8_t* w1p,
                  uint8_t* w2p) {
  const int D = d_model;
  const size_t w1rs = (size_t)D + 16, w2rs = kHC + 16;
  for (int c = 0; c < d_ff / kHC; ++c) {
    uint8_t* b1 = w1p + (size_t)c * kHC * w1rs;
    for (int r = 0; r < kHC; ++r)
      for (size_t k = 0; k < w1rs; ++k) b1[r * w1rs + k] = k < (size_t)D ? w1t[(size_t)(c * kHC + r) * D + k] : 0;
    uint8_t* b2 = w2p + (size_t)c * D * w2rs;
    for (int o = 0; o < D; ++o)
      for (size_t k = 0; k < w2rs; ++k) b2[o * w2rs + k] = k < kHC ? w2t[(size_t)o * d_ff + c * kHC + k] : 0;
  }
}

hipError_t launch_ffn_fp8(const FfnArgs& p, hipStream_t s) {
  if (!ffn_fused_supported(p.d_model, p.d_ff) || !p.ln_in_g) return hipErrorInvalidValue;
  switch (p.d_model) {
    case 64: return p.relu ? launch_fp8_d<64, true>(p, s) : launch_fp8_d<64, false>(p, s);
    case 128: return p.relu ? launch_fp8_d<128, true>(p, s) : launch_fp8_d<128, false>(p, s);
    default: return p.relu ? launch_fp8_d<256, true>(p, s) : launch_fp8_d<256, false>(p, s);
  }
}

}  // namespace mlpf
