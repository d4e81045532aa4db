// Tiled MFMA GEMM with a fused conversion prologue and fused epilogues (bias, GELU,
// residual update, head-major Q/K/V scatter). All dense products of the MLPF forward pass run
// here: embedding FFN, Q/K/V projection, attention output projection, both FFN layers and the
// output heads (first layer, with the second one optionally in the epilogue; paper Sec. 5.3).
//
// C[M][N] = op_A(A)[M][K] * W[K][N], with W stored transposed (W^T [N][Kp], the operand type) so
// that both operands are k-contiguous rows. A workgroup owns a BM x BN output tile; its waves
// (WM x WN) each own a (BM/WM) x (BN/WN) sub-tile made of 32x32 MFMA blocks. k-tiles of BK
// elements of A and W^T are staged through LDS (double buffered, one barrier per k-tile): the
// next tile's global loads are issued before the current tile's MFMAs and written to LDS after
// them. LDS rows are padded by 16 bytes so that the 32 rows read by one MFMA operand load fall
// in different banks. The epilogue is staged through the same LDS (see below).
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace mlpf {

// E_HEADS staging: 64 rows of 256 bf16 hidden units (row stride 528 bytes: 16-byte reads of 16
// consecutive rows hit distinct banks), then W2^T hi and lo, 16 rows each of the same stride.
constexpr int kHeadsRS = 528;
constexpr int kHeadsHid = 64 * kHeadsRS;

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) const void gbl_cvoid;

template <class T, int ALD, int EPI, int BM, int BN, int BK, int WM, int WN, bool PERSIST, bool DMA>
__global__ __launch_bounds__(64 * WM * WN) void gemm_kernel(const GemmArgs p) {
  using S = typename T::storage;
  constexpr int NT = 64 * WM * WN;
  constexpr int E = 16 / T::kBytes;        // operand elements per 16-byte chunk
  constexpr int C = BK / E;                // chunks per row of a k-tile
  constexpr int RS = BK * T::kBytes + 16;  // padded LDS row stride in bytes
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int FM = WTM / 32, FN = WTN / 32;
  constexpr int A_CH = BM * C, B_CH = BN * C;
  constexpr int A_PT = (A_CH + NT - 1) / NT, B_PT = (B_CH + NT - 1) / NT;
  constexpr bool A_FROM_F32 = (ALD != A_PLAIN);
  constexpr int A_BYTES = BM * RS, B_BYTES = BN * RS;
  constexpr bool kSplit = (T::kBytes == 4);
  static_assert(C % (T::kBytes == 1 ? 4 : 2) == 0 && FM >= 1 && FN >= 1, "bad tile");
  // DMA (plain A only): k-tiles of A and W^T travel by direct-to-LDS loads through kStages LDS
  // stages, unpadded rows with the 16-byte chunks of row r permuted by an XOR with swz(r) (the 8
  // rows one ds_read_b128 phase serves then hit distinct banks); the loads of k-tile kt + 2 are in
  // flight while k-tile kt is multiplied, with no registers holding them.
  constexpr bool kDma = DMA && ALD == A_PLAIN;
  constexpr int kStages = 3;
  static_assert(!(kDma && PERSIST), "DMA tiles are not persistent");
  static_assert(!kDma || ((BM * C) % NT == 0 && (BN * C) % NT == 0), "DMA tile: whole loads per wave");

  // Epilogue staging: rows of the tile, FP32, or bf16 where the output is exactly the bf16 rounding
  // of the staged value (so the rounding happens once, on the way into LDS); one pass, or one pass
  // per wave row when the full tile does not fit the main loop's LDS. E_HEADS stages bf16 rows and
  // the head's slice of W2 instead.
  constexpr bool kStageB16 = (EPI == E_QKV || EPI == E_GELU) ? sizeof(S) == 2 : EPI == E_BIAS_B;
  constexpr int SRS = BN * (kStageB16 ? 2 : 4) + 16;    // staging row stride (bytes)
  constexpr int MAIN = kDma ? kStages * (BM + BN) * C * 16 : 2 * (A_BYTES + B_BYTES);
  constexpr int PASSES = (BM * SRS <= MAIN || WM == 1) ? 1 : WM;
  constexpr int PROWS = BM / PASSES;                     // rows staged per pass
  constexpr int STAGE = EPI == E_HEADS ? kHeadsHid + 32 * kHeadsRS : PROWS * SRS;
  constexpr int SMEM = MAIN > STAGE ? MAIN : STAGE;
  static_assert(EPI != E_HEADS || (BM == 64 && BN == 256 && NT == 256), "E_HEADS tile is 64 x 256, 4 waves");
  __shared__ __attribute__((aligned(16))) char smem[SMEM];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int ntn = (p.N + BN - 1) / BN;
  int M = p.M;
  if (p.m_dev) M = min(M, max(*p.m_dev, 0));
  const int ntiles = ((M + BM - 1) / BM) * ntn;

  // Tile schedule. One tile per workgroup: xcd_remap gives each XCD a contiguous range of tiles.
  // Persistent (grid = a multiple of 8 workgroups resident at once): the tiles are cut into 8
  // contiguous ranges, one per XCD, and the workgroups of an XCD take its tiles round-robin, so
  // at any time they work on neighbouring tiles (the column tiles of the same rows, whose A rows
  // then come from that XCD's L2); the first k-tile of a workgroup's next tile is fetched before
  // the epilogue of the current one.
  int tile, tile_end, tile_step;
  if constexpr (PERSIST) {
    const int per_xcd = (ntiles + 7) / 8;
    const int x = blockIdx.x % 8, j = blockIdx.x / 8;
    tile = x * per_xcd + j;
    tile_end = min(ntiles, (x + 1) * per_xcd);
    tile_step = gridDim.x / 8;
  } else {
    tile = xcd_remap(blockIdx.x, gridDim.x);
    tile_end = min(ntiles, tile + 1);
    tile_step = 1;
  }
  if (tile >= tile_end) return;  // uniform over the workgroup
  int m0 = (tile / ntn) * BM, n0 = (tile % ntn) * BN;

  u32x4 ra[A_FROM_F32 ? 1 : A_PT];
  float raf[A_FROM_F32 ? A_PT * E : 1];
  u32x4 rb[B_PT];

  // Plain A and W^T are read with bounded buffer loads whose descriptors cover the tile's own rows
  // (columns of W): rows at or past M (columns past N) read as zeros without a compare per chunk,
  // and the byte offsets stay within the tile.
  auto load = [&](int m0, int n0, int k0) {
    if constexpr (ALD == A_PLAIN) {
      const int rows = max(0, min(BM, M - m0));
      const __amdgpu_buffer_rsrc_t ars = __builtin_amdgcn_make_buffer_rsrc(
          (void*)((const S*)p.a + (int64_t)m0 * p.lda), (short)0, rows * p.lda * (int)sizeof(S), kBufferWord3);
#pragma unroll
      for (int t = 0; t < A_PT; ++t) {
        const int c = t * NT + tid;
        if (A_CH % NT == 0 || c < A_CH)
          ra[t] = __builtin_amdgcn_raw_buffer_load_b128(
              ars, ((c / C) * p.lda + k0 + (c % C) * E) * (int)sizeof(S), 0, 0);
      }
    } else {
#pragma unroll
      for (int t = 0; t < A_PT; ++t) {
        const int c = t * NT + tid;
        const int row = c / C, ch = c % C;
        const int grow = m0 + row, kb = k0 + ch * E;
        const bool ok = (A_CH % NT == 0 || c < A_CH) && grow < M;
        if constexpr (ALD == A_SCALAR) {
          const float* ar = (const float*)p.a + (int64_t)(ok ? grow : 0) * p.lda;
#pragma unroll
          for (int e = 0; e < E; ++e) raf[t * E + e] = (ok && kb + e < p.K) ? ar[kb + e] : 0.f;
        } else {
          const f32x4* ar = (const f32x4*)((const float*)p.a + (int64_t)(ok ? grow : 0) * p.lda + kb);
#pragma unroll
          for (int e = 0; e < E / 4; ++e) {
            const f32x4 v = ok ? ar[e] : f32x4{0.f, 0.f, 0.f, 0.f};
            raf[t * E + 4 * e + 0] = v[0];
            raf[t * E + 4 * e + 1] = v[1];
            raf[t * E + 4 * e + 2] = v[2];
            raf[t * E + 4 * e + 3] = v[3];
          }
        }
      }
    }
    const int cols = max(0, min(BN, p.N - n0));
    const __amdgpu_buffer_rsrc_t brs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)((const S*)p.wt + (int64_t)n0 * p.Kp), (short)0, cols * p.Kp * (int)sizeof(S), kBufferWord3);
#pragma unroll
    for (int t = 0; t < B_PT; ++t) {
      const int c = t * NT + tid;
      if (B_CH % NT == 0 || c < B_CH)
        rb[t] = __builtin_amdgcn_raw_buffer_load_b128(
            brs, ((c / C) * p.Kp + k0 + (c % C) * E) * (int)sizeof(S), 0, 0);
    }
  };

  auto store = [&](int buf) {
    char* As = smem + buf * (A_BYTES + B_BYTES);
    char* Bs = As + A_BYTES;
#pragma unroll
    for (int t = 0; t < A_PT; ++t) {
      const int c = t * NT + tid;
      if (A_CH % NT != 0 && c >= A_CH) break;
      const int row = c / C, ch = c % C;
      u32x4 val;
      if constexpr (ALD == A_PLAIN) {
        val = ra[t];
      } else {
        val = to_chunk<T>(&raf[t * E]);
      }
      *(u32x4*)(As + row * RS + ch * 16) = val;
    }
#pragma unroll
    for (int t = 0; t < B_PT; ++t) {
      const int c = t * NT + tid;
      if (B_CH % NT != 0 && c >= B_CH) break;
      const int n = c / C, ch = c % C;
      *(u32x4*)(Bs + n * RS + ch * 16) = rb[t];
    }
  };

  const int nk = p.Kp / BK;
  const int i = lane & 31, h = lane >> 5;
  [[maybe_unused]] float amax = 0.f;  // E_GELU: largest |output| of this workgroup's tiles
  if constexpr (!kDma) load(m0, n0, 0);
  // The 16-byte chunk ch of LDS operand row r (DMA stages: permuted, unpadded rows).
  auto swz = [](int r) { return C == 4 ? (r >> 1) & 3 : (r & 7) & (C - 1); };
  auto frag = [&](const char* base, int r, int ch) -> u32x4 {
    if constexpr (kDma)
      return *(const u32x4*)(base + (r * C + (ch ^ swz(r))) * 16);
    else
      return *(const u32x4*)(base + r * RS + ch * 16);
  };
  // Direct-to-LDS loads of k-tile k0 into DMA stage st: load t of a thread fills slot t NT + tid
  // (row slot / C, position slot % C) with the chunk (position XOR swz(row)) of that row; rows past
  // M (columns past N) read the last valid one, whose products only reach discarded outputs.
  [[maybe_unused]] auto dma = [&](int st, int k0) {
    char* As = smem + st * (BM + BN) * C * 16;
    char* Bs = As + BM * C * 16;
    const S* a = (const S*)p.a;
    const S* w = (const S*)p.wt;
#pragma unroll
    for (int t = 0; t < BM * C / NT; ++t) {
      const int slot = t * NT + tid, r = slot / C, q = slot % C;
      const int row = min(m0 + r, M - 1);
      __builtin_amdgcn_global_load_lds((gbl_cvoid*)(a + (int64_t)row * p.lda + k0 + (q ^ swz(r)) * E),
                                       (lds_void*)(As + (t * NT + wave * 64) * 16), 16, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < BN * C / NT; ++t) {
      const int slot = t * NT + tid, r = slot / C, q = slot % C;
      const int col = min(n0 + r, p.N - 1);
      __builtin_amdgcn_global_load_lds((gbl_cvoid*)(w + (int64_t)col * p.Kp + k0 + (q ^ swz(r)) * E),
                                       (lds_void*)(Bs + (t * NT + wave * 64) * 16), 16, 0, 0);
    }
  };
  while (true) {
  f32x16 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = f32x16{};

  // One k-tile's products from the operand images at As and Bs.
  auto ktile = [&](const char* As, const char* Bs) {
    // FP32 operands: each k-tile sums into a fresh partial that is then added to the total, so
    // the longest chain of sequential FP32 additions is BK/2 + K/BK instead of K/2.
    f32x16 part[kSplit ? FM : 1][kSplit ? FN : 1];
    if constexpr (kSplit) {
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) part[a][b] = f32x16{};
    }
    if constexpr (T::kBytes == 1) {
      // FP8: 64-value k-groups (32x32x64 MFMA); lane half h reads the group's chunks 2h and 2h+1.
#pragma unroll
      for (int g = 0; g < C / 4; ++g) {
        u32x4 af[FM][2], bf[FN][2];
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int e = 0; e < 2; ++e)
            af[a][e] = frag(As, wm * WTM + a * 32 + i, 4 * g + 2 * h + e);
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
          for (int e = 0; e < 2; ++e)
            bf[b][e] = frag(Bs, wn * WTN + b * 32 + i, 4 * g + 2 * h + e);
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b) mma_fp8_k64(af[a][0], af[a][1], bf[b][0], bf[b][1], acc[a][b]);
      }
    } else {
#pragma unroll
    for (int g = 0; g < C / 2; ++g) {
      u32x4 af[FM], bf[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a)
        af[a] = frag(As, wm * WTM + a * 32 + i, 2 * g + h);
#pragma unroll
      for (int b = 0; b < FN; ++b)
        bf[b] = frag(Bs, wn * WTN + b * 32 + i, 2 * g + h);
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
          if constexpr (kSplit)
            mma_kg<T>(af[a], bf[b], part[a][b]);
          else
            mma_kg<T>(af[a], bf[b], acc[a][b]);
        }
    }
    }
    if constexpr (kSplit) {
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] += part[a][b];
    }
  };

  if constexpr (kDma) {
    // Stage kt % 3 holds k-tile kt. Each step waits for its own loads of k-tile kt (those of kt + 1
    // may stay in flight: the wave's vector-memory counter counts only these loads here), meets
    // the other waves at a barrier (after which every wave has loaded k-tile kt and finished
    // reading stage (kt + 2) % 3 = (kt - 1) % 3), starts k-tile kt + 2 into that stage, and
    // multiplies k-tile kt. No fence: the barrier alone orders the stages.
    constexpr int DPS = (BM + BN) * C / NT;  // direct-to-LDS loads per thread and k-tile
    constexpr int kWaitOne = (DPS & 15) | ((DPS >> 4) << 14) | (7 << 4) | (15 << 8);  // vmcnt(DPS)
    constexpr int kWaitAll = (7 << 4) | (15 << 8);                                    // vmcnt(0)
    static_assert(DPS <= 63, "vmcnt range");
    dma(0, 0);
    if (nk > 1) dma(1, BK);
    for (int kt = 0; kt < nk; ++kt) {
      // (the signal fences keep the compiler from moving LDS reads or copies across the barrier)
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (kt + 1 < nk)
        __builtin_amdgcn_s_waitcnt(kWaitOne);
      else
        __builtin_amdgcn_s_waitcnt(kWaitAll);
      __builtin_amdgcn_s_barrier();
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (kt + 2 < nk) dma((kt + 2) % kStages, (kt + 2) * BK);
      const char* As = smem + (kt % kStages) * (BM + BN) * C * 16;
      ktile(As, As + BM * C * 16);
    }
    __syncthreads();  // every wave is done with the stages before the epilogue reuses the LDS
  } else {
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) load(m0, n0, (kt + 1) * BK);
      const char* As = smem + buf * (A_BYTES + B_BYTES);
      ktile(As, As + A_BYTES);
      if (kt + 1 < nk) store(buf ^ 1);
      __syncthreads();
    }
  }
  const int next = tile + tile_step;
  if constexpr (PERSIST) {
    if (next < tile_end) load((next / ntn) * BM, (next % ntn) * BN, 0);
  }

  // Epilogue, staged through LDS so that global memory sees whole 16-byte row chunks: the waves
  // write bias + activation (FP32) into an LDS tile, then every thread moves 16-byte chunks of
  // output rows (read-modify-write of h for the residual update). In a 32x32 accumulator block,
  // lane l holds column l%32 of rows 8*(r/4) + 4*(l/32) + r%4 for r = 0..15. Tiles whose FP32
  // image does not fit the LDS of the main loop are staged in two passes (one per wave row).
  constexpr bool kResF32 = (EPI == E_BIAS || EPI == E_RESID);
  constexpr bool kResB16 = (EPI == E_BIAS_B || EPI == E_RESID_B);
  constexpr int OSZ = kResF32 ? 4 : kResB16 ? 2 : (int)sizeof(S);
  constexpr int EO = 16 / OSZ;                           // output elements per 16-byte chunk
  constexpr int CPR = BN / EO;                           // chunks per staged row
  // bf16 residual update: the h chunks of a pass are loaded before its staging, so that their
  // latency passes meanwhile (the next pass's right after this pass's last use).
  constexpr bool kPrefH = (EPI == E_RESID_B);
  constexpr int RPP = (PROWS * CPR + NT - 1) / NT;       // chunks per thread and pass
  [[maybe_unused]] u32x4 hv[kPrefH ? RPP : 1];
  [[maybe_unused]] auto hload = [&](int pass) {
#pragma unroll
    for (int q = 0; q < RPP; ++q) {
      const int c = tid + q * NT;
      const int row = m0 + pass * PROWS + c / CPR, col = n0 + (c % CPR) * EO;
      hv[q] = (c < PROWS * CPR && row < M && col < p.N)
                  ? *(const u32x4*)((const __bf16*)p.out + (int64_t)row * p.ldo + col)
                  : u32x4{0, 0, 0, 0};
    }
  };
  if constexpr (kPrefH) hload(0);
#pragma unroll
  for (int pass = 0; pass < PASSES; ++pass) {
    if (PASSES == 1 || wm == pass) {
#pragma unroll
      for (int a = 0; a < FM; ++a) {
#pragma unroll
        for (int b = 0; b < FN; ++b) {
          const int lcol = wn * WTN + b * 32 + i;
          const int col = n0 + lcol;
          const float bias = (p.bias && col < p.N) ? p.bias[col] : 0.f;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int lrow = (PASSES == 1 ? wm * WTM : 0) + a * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
            float v = (T::kBytes == 1 ? acc[a][b][r] * p.acc_scale : acc[a][b][r]) + bias;
            if constexpr (EPI == E_GELU) {
              // (FP32: the erf form; bf16 and FP8 outputs: the logistic form, see gelu_fast)
              v = p.relu ? fmaxf(v, 0.f) : T::kBytes == 4 ? gelu_erf(v) : gelu_fast(v);
              if (m0 + pass * PROWS + lrow < M && col < p.N) amax = fmaxf(amax, fabsf(v));
            }
            if constexpr (EPI == E_HEADS) {  // the hidden layer, bf16 rows of kHeadsRS bytes
              *(__bf16*)(smem + lrow * kHeadsRS + lcol * 2) = (__bf16)(p.relu ? fmaxf(v, 0.f) : gelu_fast(v));
            } else if constexpr (kStageB16) {
              if constexpr (EPI == E_QKV) v *= col < p.d ? p.q_scale : 1.f;  // Q pre-scaled
              *(__bf16*)(smem + lrow * SRS + lcol * 2) = (__bf16)v;
            } else {
              *(float*)(smem + lrow * SRS + lcol * 4) = v;
            }
          }
        }
      }
    }
    if constexpr (EPI == E_HEADS) {
      // Second layer of head k = head0 + n0 / 256 on the 64 x 256 bf16 hidden tile staged above:
      // out^T [16 outputs (zero-padded)][64 rows] = W2_k^T [16][256] U^T [256][64] with
      // v_mfma_f32_16x16x32_bf16 (lane l: output / row l % 16, k = 8 (l / 16) .. + 7 of each
      // 32-wide k-step). W2 is FP32: it enters as hi + lo, hi = bf16(w), lo = bf16(w - hi), two
      // products into the same FP32 sums (|w - hi - lo| <= 2^-18 |w|). Wave w owns rows 16 w ..
      // 16 w + 15.
      // Output columns of head k: five heads cls 0..5, pT 6, eta 7, phi 8..9, E 10; six heads
      // binary 0, pid 1..5, then the same four.
      const int k = p.head0 + n0 / 256;
      const int k6 = p.heads6 ? k : k + 1;  // index in the six-head order (k > 0 for five heads)
      const int c0 = (!p.heads6 && k == 0) ? 0 : k6 == 0 ? 0 : k6 == 1 ? 1 : k6 + 4 + (k6 == 5);
      const int wid = (!p.heads6 && k == 0) ? 6 : k6 == 0 ? 1 : k6 == 1 ? 5 : k6 == 4 ? 2 : 1;
      char* w2s = smem + kHeadsHid;  // [2 (hi, lo)][16][kHeadsRS]
      {
        const int j = tid;  // hidden unit (NT == 256)
#pragma unroll
        for (int o = 0; o < 16; ++o) {
          const float w = o < wid ? p.w2[j * 11 + c0 + o] : 0.f;
          const __bf16 hi = (__bf16)w;
          const __bf16 lo = (__bf16)(w - (float)hi);
          *(__bf16*)(w2s + o * kHeadsRS + 2 * j) = hi;
          *(__bf16*)(w2s + (16 + o) * kHeadsRS + 2 * j) = lo;
        }
      }
      __syncthreads();
      const int r16 = lane & 15, kq = lane >> 4;
      const char* ub = smem + (16 * wave + r16) * kHeadsRS + 16 * kq;
      const char* wh = w2s + r16 * kHeadsRS + 16 * kq;
      const char* wl = wh + 16 * kHeadsRS;
      f32x4 o4 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int st = 0; st < 8; ++st) {
        const bf16x8 u = __builtin_bit_cast(bf16x8, *(const u32x4*)(ub + 64 * st));
        const bf16x8 a_hi = __builtin_bit_cast(bf16x8, *(const u32x4*)(wh + 64 * st));
        const bf16x8 a_lo = __builtin_bit_cast(bf16x8, *(const u32x4*)(wl + 64 * st));
        o4 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi, u, o4, 0, 0, 0);
        o4 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_lo, u, o4, 0, 0, 0);
      }
      // Lane holds row 16 w + l % 16 and outputs 4 (l / 16) + e.
      const int row = m0 + 16 * wave + r16;
      if (row < M) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int o = 4 * kq + e;
          if (o < wid) p.hout[(int64_t)row * 11 + c0 + o] = o4[e];
        }
      }
      continue;
    }
    __syncthreads();
    if constexpr (kPrefH) {
#pragma unroll
      for (int q = 0; q < RPP; ++q) {
        const int c = tid + q * NT;
        if (PROWS * CPR % NT != 0 && c >= PROWS * CPR) break;
        const int lrow = c / CPR, lc = (c % CPR) * EO;
        const int row = m0 + pass * PROWS + lrow, col = n0 + lc;
        if (row < M && col < p.N) {
          const float* src = (const float*)(smem + lrow * SRS + lc * 4);
          const u32x4 o = hv[q];
          const f32x4 v0 = *(const f32x4*)src + f32x4{__uint_as_float(o[0] << 16), __uint_as_float(o[0] & 0xffff0000u),
                                                      __uint_as_float(o[1] << 16), __uint_as_float(o[1] & 0xffff0000u)};
          const f32x4 v1 = *(const f32x4*)(src + 4) + f32x4{__uint_as_float(o[2] << 16), __uint_as_float(o[2] & 0xffff0000u),
                                                            __uint_as_float(o[3] << 16), __uint_as_float(o[3] & 0xffff0000u)};
          const u32x2 lo = pack_bf16x4(v0[0], v0[1], v0[2], v0[3]);
          const u32x2 hi = pack_bf16x4(v1[0], v1[1], v1[2], v1[3]);
          *(u32x4*)((__bf16*)p.out + (int64_t)row * p.ldo + col) = u32x4{lo[0], lo[1], hi[0], hi[1]};
        }
      }
      if (pass + 1 < PASSES) hload(pass + 1);
      if (PASSES > 1 && pass + 1 < PASSES) __syncthreads();
      continue;
    }
    for (int c = tid; c < PROWS * CPR; c += NT) {
      const int lrow = c / CPR, lc = (c % CPR) * EO;
      const int row = m0 + pass * PROWS + lrow, col = n0 + lc;
      const bool live = row < M && col < p.N;
      [[maybe_unused]] float ss = 0.f;  // E_QKV with knorm: sum of squares of this K chunk
      if (live) {
      const float* src = (const float*)(smem + lrow * SRS + lc * (kStageB16 ? 2 : 4));
      if constexpr (kResF32) {
        f32x4 v = *(const f32x4*)src;
        f32x4* dst = (f32x4*)((float*)p.out + (int64_t)row * p.ldo + col);
        if constexpr (EPI == E_RESID) v += *dst;
        *dst = v;
      } else if constexpr (kResB16) {  // E_BIAS_B (E_RESID_B takes the loop above): staged as bf16
        *(u32x4*)((__bf16*)p.out + (int64_t)row * p.ldo + col) = *(const u32x4*)src;
      } else {
        [[maybe_unused]] float qs = 1.f;
        S* dst;
        if constexpr (EPI == E_QKV) {
          const int which = col / p.d, rem = col % p.d;
          const int hh = rem / p.dh, cc = rem % p.dh;
          dst = (S*)(which == 0 ? p.q : which == 1 ? p.k : p.v) + (int64_t)hh * p.hstride +
                (int64_t)row * p.dh + cc;
          qs = which == 0 ? p.q_scale : 1.f;
        } else {
          dst = (S*)p.out + (int64_t)row * p.ldo + col;
        }
        // Q, K and V are written with non-temporal stores: they are read back by the next kernel
        // from memory, and streaming them through L2 would evict the tiles of W every workgroup
        // re-reads.
        if constexpr (sizeof(S) == 4) {
          const f32x4 v = *(const f32x4*)src;
          if constexpr (EPI == E_QKV)
            __builtin_nontemporal_store(v * qs, (f32x4*)dst);
          else
            *(f32x4*)dst = v * qs;
        } else if constexpr (sizeof(S) == 2) {  // staged as bf16 (Q already scaled)
          const u32x4 w = *(const u32x4*)src;
          if constexpr (EPI == E_QKV)
            __builtin_nontemporal_store(w, (u32x4*)dst);
          else
            *(u32x4*)dst = w;
          if constexpr (EPI == E_QKV) {
            if (p.knorm && col >= p.d && col < 2 * p.d) {
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const float a = __uint_as_float(w[e] << 16), b = __uint_as_float(w[e] & 0xffff0000u);
                ss = fmaf(a, a, fmaf(b, b, ss));
              }
            }
          }
        } else {
          u32x4 o;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const f32x4 v = *(const f32x4*)(src + 4 * q);
            o[q] = pack_fp8x4(v[0] * p.out_scale, v[1] * p.out_scale, v[2] * p.out_scale,
                              v[3] * p.out_scale);
          }
          *(u32x4*)dst = o;
        }
      }
      }
      if constexpr (EPI == E_QKV && sizeof(S) == 2) {
        // Squared norm of each (row, head) of K from its bf16 values: the dh/8 chunks of one head
        // are consecutive threads (the tile's columns start on a head boundary).
        if (p.knorm) {
          ss += xor_lane(ss, 1);
          if (p.dh == 32) ss += xor_lane(ss, 2);
          const int rem = col - p.d;
          if (live && rem >= 0 && rem < p.d && rem % p.dh == 0)
            p.knorm[(int64_t)(rem / p.dh) * (p.hstride / p.dh) + row] = ss;
        }
      }
    }
    if (PASSES > 1 && pass + 1 < PASSES) __syncthreads();
  }
  if (!PERSIST || next >= tile_end) break;
  __syncthreads();  // the staging reads are done before the next tile's first LDS store
  tile = next;
  m0 = (tile / ntn) * BM;
  n0 = (tile % ntn) * BN;
  }
  if constexpr (EPI == E_GELU) {
    if (p.amax) {
      amax = wave_max(amax);
      if (lane == 0) atomic_max_nonneg(p.amax, amax);
    }
  }
}

namespace {

constexpr GemmTile kTiles[] = {
    {64, 64, 2, 2, 128, 0},
    {128, 64, 2, 2, 128, 0},
    {128, 128, 2, 2, 128, 0},
    {64, 128, 2, 2, 128, 0},
    {256, 128, 2, 2, 128, 0},  // wave tile 128x64: fewer LDS bytes per MFMA
    {128, 256, 2, 2, 128, 0},  // wave tile 64x128
    // 64-byte k-tiles: half the LDS per workgroup, so more workgroups per CU hide load latency
    {128, 128, 2, 2, 64, 0},
    {128, 64, 2, 2, 64, 0},
    {64, 128, 2, 2, 64, 0},
    // persistent workgroups (next tile's first k-tile fetched during the epilogue)
    {128, 128, 2, 2, 64, 1},
    {128, 64, 2, 2, 64, 1},
    {64, 128, 2, 2, 64, 1},
    {128, 128, 2, 2, 128, 1},
    // 64 rows x 256 columns, 1 x 4 waves: whole 256-wide rows per workgroup (fused output heads)
    {64, 256, 1, 4, 64, 0},
    // 8 waves with 64 x 64 wave tiles, k-tiles by direct-to-LDS loads through three LDS stages
    // (plain A operands; a converted FP32 A runs the shape double buffered through registers): the
    // larger tiles cut the L2 reads of A and W^T (each row of one is read once per tile of the
    // other), and the loads need no staging registers
    {128, 256, 2, 4, 64, 2},
    {256, 128, 4, 2, 64, 2},
};

// Workgroups of one kernel that fit on the device at once (the grid of a persistent launch). The
// result only sizes the grid: the tile schedule is correct for any grid that is a multiple of 8.
template <class K>
int resident_workgroups(K kernel, int threads) {
  static int cached = 0;
  if (cached > 0) return cached;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu <= 0)
    return cus * 2;
  cached = cus * per_cu;
  return cached;
}

template <class T, int ALD, int EPI, int BM, int BN, int WM, int WN, int BKB = 128, bool PERSIST = false,
          bool DMA = false>
hipError_t launch_t(const GemmArgs& p, hipStream_t s) {
  constexpr int BK = BKB / T::kBytes;  // BKB bytes of each row per k-tile
  if (p.Kp % BK != 0 || p.N % 16 != 0) return hipErrorInvalidValue;
  const int gm = (p.M + BM - 1) / BM, gn = (p.N + BN - 1) / BN;
  int64_t grid = (int64_t)gm * gn;
  if (grid == 0) return hipSuccess;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  auto kernel = gemm_kernel<T, ALD, EPI, BM, BN, BK, WM, WN, PERSIST, DMA>;
  if constexpr (PERSIST) {
    const int res = std::max(8, resident_workgroups(kernel, 64 * WM * WN));
    grid = std::min<int64_t>((grid + 7) / 8 * 8, res / 8 * 8);
  }
  hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(64 * WM * WN), 0, s, p);
  return hipGetLastError();
}

template <class T, int ALD, int EPI>
hipError_t launch_tile(int tile, const GemmArgs& p, hipStream_t s) {
  switch (tile) {
    case 0: return launch_t<T, ALD, EPI, 64, 64, 2, 2>(p, s);
    case 1: return launch_t<T, ALD, EPI, 128, 64, 2, 2>(p, s);
    case 2: return launch_t<T, ALD, EPI, 128, 128, 2, 2>(p, s);
    case 3: return launch_t<T, ALD, EPI, 64, 128, 2, 2>(p, s);
    case 4: return launch_t<T, ALD, EPI, 256, 128, 2, 2>(p, s);
    case 5: return launch_t<T, ALD, EPI, 128, 256, 2, 2>(p, s);
    case 6: return launch_t<T, ALD, EPI, 128, 128, 2, 2, 64>(p, s);
    case 7: return launch_t<T, ALD, EPI, 128, 64, 2, 2, 64>(p, s);
    case 8: return launch_t<T, ALD, EPI, 64, 128, 2, 2, 64>(p, s);
    case 9: return launch_t<T, ALD, EPI, 128, 128, 2, 2, 64, true>(p, s);
    case 10: return launch_t<T, ALD, EPI, 128, 64, 2, 2, 64, true>(p, s);
    case 11: return launch_t<T, ALD, EPI, 64, 128, 2, 2, 64, true>(p, s);
    case 12: return launch_t<T, ALD, EPI, 128, 128, 2, 2, 128, true>(p, s);
    case 13: return launch_t<T, ALD, EPI, 64, 256, 1, 4, 64>(p, s);
    case 14: return launch_t<T, ALD, EPI, 128, 256, 2, 4, 64, false, true>(p, s);
    case 15: return launch_t<T, ALD, EPI, 256, 128, 4, 2, 64, false, true>(p, s);
    default: return hipErrorInvalidValue;
  }
}

template <class T>
hipError_t launch_prec(ALoad aload, Epi epi, int tile, const GemmArgs& p, hipStream_t s) {
  // Only the combinations the forward pass uses are instantiated.
  if (aload == A_SCALAR && epi == E_GELU) return launch_tile<T, A_SCALAR, E_GELU>(tile, p, s);
  if (aload == A_PLAIN && epi == E_BIAS) return launch_tile<T, A_PLAIN, E_BIAS>(tile, p, s);
  if (aload == A_PLAIN && epi == E_QKV) return launch_tile<T, A_PLAIN, E_QKV>(tile, p, s);
  if (aload == A_PLAIN && epi == E_RESID) return launch_tile<T, A_PLAIN, E_RESID>(tile, p, s);
  if (aload == A_PLAIN && epi == E_GELU) return launch_tile<T, A_PLAIN, E_GELU>(tile, p, s);
  if constexpr (!std::is_same_v<T, F32>) {
    if (aload == A_PLAIN && epi == E_HEADS) {
      if (tile != 13 || p.N % 256 != 0 || !p.w2 || !p.hout) return hipErrorInvalidValue;
      return launch_t<T, A_PLAIN, E_HEADS, 64, 256, 1, 4, 64>(p, s);
    }
    if (aload == A_PLAIN && epi == E_BIAS_B) return launch_tile<T, A_PLAIN, E_BIAS_B>(tile, p, s);
    if (aload == A_PLAIN && epi == E_RESID_B) return launch_tile<T, A_PLAIN, E_RESID_B>(tile, p, s);
  }
  if (aload == A_F32 && epi == E_GELU) return launch_tile<T, A_F32, E_GELU>(tile, p, s);
  return hipErrorInvalidValue;
}

}  // namespace

int gemm_num_tiles() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }
GemmTile gemm_tile(int id) { return kTiles[id]; }

hipError_t launch_gemm(Prec prec, ALoad aload, Epi epi, int tile, const GemmArgs& p,
                       hipStream_t s) {
  if (prec == P_F32) return launch_prec<F32>(aload, epi, tile, p, s);
  if (prec == P_BF16) return launch_prec<BF16>(aload, epi, tile, p, s);
  if (prec == P_FP8) {
    // FP8 runs the two FFN products only (operands quantised by their producers).
    if (aload == A_PLAIN && epi == E_GELU) return launch_tile<FP8, A_PLAIN, E_GELU>(tile, p, s);
    if (aload == A_PLAIN && epi == E_RESID) return launch_tile<FP8, A_PLAIN, E_RESID>(tile, p, s);
    if (aload == A_PLAIN && epi == E_RESID_B) return launch_tile<FP8, A_PLAIN, E_RESID_B>(tile, p, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace mlpf
