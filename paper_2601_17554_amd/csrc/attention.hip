// Masked variable-length multi-head self-attention with online softmax (paper Eq. 4, computed
// exactly as the FlashAttention kernel the paper uses does: tiled, never materialising A).
//
// One workgroup = one work item (event, head, block of 32*NW*QB queries); each wave owns QB blocks
// of 32 queries, which share every K and V fragment the wave reads from LDS.
// Keys are the event's own valid elements only, so events never see each other and padding rows
// are never keys. K and V tiles of KT keys are staged through LDS (double buffered) and shared by
// the workgroup's waves; V is transposed while it is written to LDS.
//
// The scores are computed transposed, S^T = K Q^T, with 32x32 MFMAs: lane l then holds, for its
// query l%32, the scores of 16 keys of each 32-key block (keys 8*(r/4) + 4*(l/32) + r%4 in register
// r). The row maximum is one in-lane reduction plus one exchange with lane l^32, and the
// probabilities P^T are already in the layout of the B operand of the second product,
// O^T = V^T P^T, so P never leaves registers. Softmax statistics are FP32; scores are in log2
// units because Q was pre-scaled by log2(e)/sqrt(d_head), so exp2 is used.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace mlpf {

// Exchange with lane l^32 (the other half holding the same query): v_permlane32_swap.
__device__ __forceinline__ float other_half(float x) {
  const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  // sw[0] holds x of lane l%32 in every lane, sw[1] x of lane l%32 + 32.
  const float lo = __uint_as_float(sw[0]), hi = __uint_as_float(sw[1]);
  return (threadIdx.x & 32) ? lo : hi;
}

// -x as three bf16 values packed for one lane half of a 32x32x16 MFMA operand: hi + mid + lo
// represents any normal FP32 value exactly (3 x 8 significant bits), and the MFMA adds the three
// products (each exact) in FP32.
__device__ __forceinline__ u32x4 neg_split3(float x) {
  const __bf16 hi = (__bf16)(-x);
  const float r1 = -x - (float)hi;
  const __bf16 mid = (__bf16)r1;
  const __bf16 lo = (__bf16)(r1 - (float)mid);
  const uint32_t a = __builtin_bit_cast(uint16_t, hi), b = __builtin_bit_cast(uint16_t, mid);
  const uint32_t c = __builtin_bit_cast(uint16_t, lo);
  return u32x4{a | (b << 16), c, 0, 0};
}

template <class T, int DH, int NW, int KT, int QB>
__global__ __launch_bounds__(NW * 64) void attn_kernel(const AttnArgs p) {
  using S = typename T::storage;
  constexpr int NT = NW * 64;
  constexpr int SZ = T::kBytes;
  constexpr bool kBF16 = (SZ == 2);
  constexpr int E = 16 / SZ;              // elements per 16-byte chunk
  constexpr int KRS = DH * SZ + 16;       // LDS row stride of the K tile [KT][DH]
  constexpr int VRS = KT * SZ + 16;       // LDS row stride of the V^T tile [DH][KT]
  constexpr int K_BYTES = KT * KRS, V_BYTES = DH * VRS;
  constexpr int CH_ROW = DH / E;          // chunks per K or V row
  constexpr int NCH = KT * CH_ROW;        // chunks per tile
  constexpr int PT = (NCH + NT - 1) / NT;
  constexpr int NB = KT / 32;             // 32-key blocks per tile
  constexpr int QKG = DH / (2 * E);       // k-groups of the QK^T product
  static_assert(KT % 32 == 0 && DH % (2 * E) == 0 && DH <= 32, "bad attention shape");

  __shared__ __attribute__((aligned(16))) char smem[2 * (K_BYTES + V_BYTES)];

  if ((int)blockIdx.x >= min(*p.n_items, p.cap_items)) return;
  const int ev = p.items[2 * blockIdx.x], code = p.items[2 * blockIdx.x + 1];
  const int head = code & 255, qtile = code >> 8;
  const int start = p.ev_start[ev], n = p.ev_n[ev];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 31, h = lane >> 5;

  const S* qb = (const S*)p.q + (int64_t)head * p.hstride + (int64_t)start * DH;
  const S* kb = (const S*)p.k + (int64_t)head * p.hstride + (int64_t)start * DH;
  const S* vb = (const S*)p.v + (int64_t)head * p.hstride + (int64_t)start * DH;

  // This wave's QB blocks of 32 queries.
  int qi[QB];
  u32x4 qr[QB][QKG];
#pragma unroll
  for (int j = 0; j < QB; ++j) {
    qi[j] = (qtile * NW + wave) * (32 * QB) + 32 * j + i;
#pragma unroll
    for (int c = 0; c < QKG; ++c)
      qr[j][c] = qi[j] < n ? *(const u32x4*)(qb + (int64_t)qi[j] * DH + (2 * c + h) * E)
                           : u32x4{0, 0, 0, 0};
  }

  // K and V of this (event, head) are one contiguous run of n rows each. Buffer loads with the run's
  // byte length as the bound return zeros past the last key, so the tile loads need no masks.
  const int run_bytes = n * DH * SZ;
  const __amdgpu_buffer_rsrc_t krs = __builtin_amdgcn_make_buffer_rsrc((void*)kb, (short)0, run_bytes, kBufferWord3);
  const __amdgpu_buffer_rsrc_t vrs = __builtin_amdgcn_make_buffer_rsrc((void*)vb, (short)0, run_bytes, kBufferWord3);
  u32x4 rk[PT], rv[PT];
  auto load = [&](int kt0) {
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      const int c = t * NT + tid;
      const int r = c / CH_ROW, ch = c % CH_ROW;
      const int off = (kt0 + r) * (DH * SZ) + ch * 16;
      rk[t] = __builtin_amdgcn_raw_buffer_load_b128(krs, off, 0, 0);
      rv[t] = __builtin_amdgcn_raw_buffer_load_b128(vrs, off, 0, 0);
    }
  };
  auto store = [&](int buf) {
    char* Ks = smem + buf * (K_BYTES + V_BYTES);
    char* Vs = Ks + K_BYTES;
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      const int c = t * NT + tid;
      if (NCH % NT != 0 && c >= NCH) break;
      const int r = c / CH_ROW, ch = c % CH_ROW;
      *(u32x4*)(Ks + r * KRS + ch * 16) = rk[t];
      if constexpr (SZ == 4) {
#pragma unroll
        for (int e = 0; e < 4; ++e) *(uint32_t*)(Vs + (ch * 4 + e) * VRS + r * 4) = rv[t][e];
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          *(uint16_t*)(Vs + (ch * 8 + e) * VRS + r * 2) = (uint16_t)(rv[t][e >> 1] >> (16 * (e & 1)));
      }
    }
  };

  // Per-lane softmax state of each query block: m = running maximum of the scores (log2 units;
  // BF16: the offset the scores are computed against), l = partial row sum over this lane's keys
  // (the two lane halves are added at the end), oacc = O^T.
  float m_run[QB], l_run[QB];
  f32x16 oacc[QB];
  [[maybe_unused]] u32x4 qaug[QB];  // BF16: split of -m_run (lanes of half 0)
#pragma unroll
  for (int j = 0; j < QB; ++j) {
    m_run[j] = kBF16 ? 0.f : -INFINITY;
    l_run[j] = 0.f;
    oacc[j] = f32x16{};
    qaug[j] = u32x4{0, 0, 0, 0};
  }
  // BF16: the constant A operand (1, 1, 1, 0, ...) in the lanes of k-slots 0..7 (half 0).
  [[maybe_unused]] const u32x4 kaug = h == 0 ? u32x4{0x3F803F80u, 0x3F80u, 0, 0} : u32x4{0, 0, 0, 0};

  auto tile = [&](const int t, const auto masked_tag) {
    constexpr bool kMasked = decltype(masked_tag)::value;
    const int kt0 = t * KT;
    const char* Ks = smem + (t & 1) * (K_BYTES + V_BYTES);
    const char* Vs = Ks + K_BYTES;

    // K fragments of the tile, shared by the wave's query blocks.
    u32x4 ka[NB][QKG];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int c = 0; c < QKG; ++c) ka[b][c] = *(const u32x4*)(Ks + (32 * b + i) * KRS + (2 * c + h) * 16);

    // S^T = K Q^T for each query block and 32-key block (BF16: minus the current offset m, folded
    // into the product as an extra k-group: constant rows (1, 1, 1) times the exact 3-term bf16
    // split of -m).
    f32x16 s[QB][NB];
    auto scores = [&](const int j) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        s[j][b] = f32x16{};
        if constexpr (kBF16) mma_kg<T>(kaug, qaug[j], s[j][b]);
#pragma unroll
        for (int c = 0; c < QKG; ++c) mma_kg<T>(ka[b][c], qr[j][c], s[j][b]);
        if constexpr (kMasked) {
#pragma unroll
          for (int r = 0; r < 16; ++r)
            if (kt0 + 32 * b + 8 * (r >> 2) + 4 * h + (r & 3) >= n) s[j][b][r] = -INFINITY;
        }
      }
    };
    float alpha[QB];
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      scores(j);
      float mx = -INFINITY;
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) mx = fmaxf(mx, s[j][b][r]);
      mx = fmaxf(mx, other_half(mx));  // finite: every tile holds a valid key
      if constexpr (kBF16) {
        // mx is relative to the offset. The maximum grows on few tiles after the first: only then
        // move the offset, recompute the scores against it (MFMA work, not a VALU subtraction per
        // score) and rescale O and l; the branch is wave-uniform.
        alpha[j] = 1.f;
        if (t == 0 || __any(mx > 0.f)) {
          const float m_new = (t == 0) ? m_run[j] + mx : m_run[j] + fmaxf(mx, 0.f);
          // Nothing is accumulated before the first tile: its factor is 0 (the offset starts at 0,
          // not at -inf, so exp2(m_run - m_new) would overflow for maxima below -128).
          const float a = (t == 0) ? 0.f : __builtin_amdgcn_exp2f(m_run[j] - m_new);
          m_run[j] = m_new;
          qaug[j] = h == 0 ? neg_split3(m_new) : u32x4{0, 0, 0, 0};
          l_run[j] *= a;
#pragma unroll
          for (int r = 0; r < 16; ++r) oacc[j][r] *= a;
          scores(j);
        }
      } else {
        const float m_new = fmaxf(m_run[j], mx);
        alpha[j] = __builtin_amdgcn_exp2f(m_run[j] - m_new);  // 0 on the first tile
        m_run[j] = m_new;
      }
    }

    if constexpr (kBF16) {
      // P = exp2(S') in FP32, packed to bf16 for the PV product; l sums the packed values, so
      // numerator and denominator of O = sum P v / sum P carry the same rounded weights.
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          // O^T += V^T P^T: row dh = l%32 of V^T, keys matching the P^T register order; the V^T
          // fragment is shared by the query blocks.
          u32x4 va = u32x4{0, 0, 0, 0};
          if (i < DH) {
            const u32x2 v0 = *(const u32x2*)(Vs + i * VRS + (32 * b + 16 * c + 4 * h) * 2);
            const u32x2 v1 = *(const u32x2*)(Vs + i * VRS + (32 * b + 16 * c + 8 + 4 * h) * 2);
            va = u32x4{v0[0], v0[1], v1[0], v1[1]};
          }
#pragma unroll
          for (int j = 0; j < QB; ++j) {
            u32x4 pb;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              const float e0 = __builtin_amdgcn_exp2f(s[j][b][8 * c + 4 * q + 0]);
              const float e1 = __builtin_amdgcn_exp2f(s[j][b][8 * c + 4 * q + 1]);
              const float e2 = __builtin_amdgcn_exp2f(s[j][b][8 * c + 4 * q + 2]);
              const float e3 = __builtin_amdgcn_exp2f(s[j][b][8 * c + 4 * q + 3]);
              const u32x2 pk = pack_bf16x4(e0, e1, e2, e3);
              l_run[j] = add_bf16x4(e0, e1, e2, e3, l_run[j]);
              pb[2 * q] = pk[0];
              pb[2 * q + 1] = pk[1];
            }
            mma_kg<T>(va, pb, oacc[j]);
          }
        }
      }
    } else {
      // FP32: P = exp2(S - m); the tile's PV product goes to a fresh partial first (shorter
      // sequential addition chains over long events).
      f32x16 pv[QB];
#pragma unroll
      for (int j = 0; j < QB; ++j) {
        float ls = 0.f;
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const float e = __builtin_amdgcn_exp2f(s[j][b][r] - m_run[j]);
            s[j][b][r] = e;
            ls += e;
          }
        l_run[j] = l_run[j] * alpha[j] + ls;
        pv[j] = f32x16{};
      }
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const u32x4 va = (i < DH) ? *(const u32x4*)(Vs + i * VRS + (32 * b + 8 * c + 4 * h) * 4)
                                    : u32x4{0, 0, 0, 0};
#pragma unroll
          for (int j = 0; j < QB; ++j) {
            const u32x4 pb = {__float_as_uint(s[j][b][4 * c + 0]), __float_as_uint(s[j][b][4 * c + 1]),
                              __float_as_uint(s[j][b][4 * c + 2]), __float_as_uint(s[j][b][4 * c + 3])};
            mma_kg<T>(va, pb, pv[j]);
          }
        }
#pragma unroll
      for (int j = 0; j < QB; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) oacc[j][r] = oacc[j][r] * alpha[j] + pv[j][r];
    }
  };

  const int nkt = (n + KT - 1) / KT;
  if (nkt > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  // Full tiles, then the last partial tile (the only one that needs the key mask).
  const int nfull = n / KT;
  for (int t = 0; t < nfull; ++t) {
    if (t + 1 < nkt) load((t + 1) * KT);
    tile(t, std::false_type{});
    if (t + 1 < nkt) store((t + 1) & 1);
    __syncthreads();
  }
  if (nfull < nkt) tile(nfull, std::true_type{});

  // O = O^T / l. Lane l holds dh = 8c + 4*(l/32) + (0..3) of query l%32 in registers 4c..4c+3.
#pragma unroll
  for (int j = 0; j < QB; ++j) {
    const float l_tot = l_run[j] + other_half(l_run[j]);
    if (qi[j] < n) {
      const float inv = 1.0f / l_tot;
      S* orow = (S*)p.o + (int64_t)(start + qi[j]) * p.d + head * DH;
#pragma unroll
      for (int c = 0; c < DH / 8; ++c) {
        const float a0 = oacc[j][4 * c] * inv, a1 = oacc[j][4 * c + 1] * inv;
        const float a2 = oacc[j][4 * c + 2] * inv, a3 = oacc[j][4 * c + 3] * inv;
        if constexpr (SZ == 4) {
          *(f32x4*)(orow + 8 * c + 4 * h) = f32x4{a0, a1, a2, a3};
        } else {
          *(u32x2*)(orow + 8 * c + 4 * h) = pack_bf16x4(a0, a1, a2, a3);
        }
      }
    }
  }
}

// BF16 attention without running maxima. The softmax of Eq. 4 is invariant under a per-query shift
// of the scores; any shift m_q >= max_k s_qk keeps every exponential at or below 1, and one that is
// not far above the maximum keeps the largest exponentials in the normal FP32 range. The kernel takes
// the Cauchy-Schwarz bound m_q = |q| max_k |k| (slightly enlarged to cover the rounding of the FP32
// dot products), with max_k |k|^2 read from a per-(head, row) table of squared key norms. The shift
// enters the QK^T MFMA as its C operand (16 accumulator registers holding -m_q), so each score costs
// one exp2 and half a dot2 into the row sum, with no maximum, comparison or rescaling in the key
// loop. If the bound exceeds the true maximum by more than 96 (log2 units) for some query, its row
// sum would lose precision; the workgroup then computes the exact maxima in an extra pass over the
// keys and runs the key loop again with them.
//
// Key loop: 32-key blocks, software pipelined (the QK^T product of block b+1 is issued before the
// exponentials of block b, with the two score sets in alternating registers, and its K fragments
// were read from LDS a step earlier). PIPE false drops the look-ahead: each block is scored
// and consumed in one step, and the score set fewer in registers lets three waves share a SIMD,
// whose interleaving then hides the MFMA latency (the faster form at d_head 32). K and V stages of
// 32*G keys rotate through three LDS slots: while stage s is consumed, stage s+1 is resident (the
// look-ahead product reads it) and stage s+2 travels from global memory in registers; one barrier
// per stage. Each wave owns QB blocks of 32 queries. V stays row-major in LDS (one 16-byte store
// per chunk); the V^T operand of O^T = V^T P^T is read with the transposing ds_read_b64_tr_b16: in
// each 16-lane group, lane j receives element j%4 of the 8-byte chunks addressed by lanes j/4,
// j/4+4, j/4+8 and j/4+12 of the group, so lane s addresses row (key) s/4 and dh columns
// 4(s%4)..4(s%4)+3 and every lane gets one dh column of four consecutive keys.
template <int DH, int NW, int G, int QB, int OCC, bool PIPE>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(OCC)))
void attn_bf16_kernel(const AttnArgs p) {
  constexpr int NT = NW * 64;
  constexpr int KEYS = 32 * G;        // keys per stage
  constexpr int KRS = DH * 2 + 16;    // LDS row stride of K [KEYS][DH]
  constexpr int VRS = DH * 2 + 32;    // LDS row stride of V [KEYS][DH]: the 4 rows x 32 bytes a
                                      // transposing read touches per lane group hit distinct banks
  constexpr int K_BYTES = KEYS * KRS, V_BYTES = KEYS * VRS, SLOT = K_BYTES + V_BYTES;
  constexpr int CH_ROW = DH / 8;      // 16-byte chunks per K or V row
  constexpr int NCH = KEYS * CH_ROW;  // chunks per stage and matrix
  constexpr int PT = (NCH + NT - 1) / NT;
  constexpr int QKG = DH / 16;        // k-groups of the QK^T product
  static_assert((DH == 16 || DH == 32) && G % 2 == 0, "bad attention shape");

  __shared__ __attribute__((aligned(16))) char smem[3 * SLOT];

  // Workgroup b runs work item b % n_it over key range b / n_it of the event (split-major).
  const int n_it = min(*p.n_items, p.cap_items);
  if ((int)blockIdx.x >= n_it * p.ksplit) return;
  const int item = (int)blockIdx.x % n_it, split = (int)blockIdx.x / n_it;
  const int ev = p.items[2 * item], code = p.items[2 * item + 1];
  const int head = code & 255, qtile = code >> 8;
  const int start = p.ev_start[ev], n = p.ev_n[ev];  // n queries; the keys are a range of them:
  const int nbs = (((n + 31) >> 5) + p.ksplit - 1) / p.ksplit;  // 32-key blocks per split
  const int k0 = 32 * nbs * split;                              // this split's first key
  const int nk = min(max(n - k0, 0), 32 * nbs);                 // and its key count

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 31, h = lane >> 5;

  const __bf16* qb = (const __bf16*)p.q + (int64_t)head * p.hstride + (int64_t)start * DH;
  const __bf16* kb = (const __bf16*)p.k + (int64_t)head * p.hstride + (int64_t)(start + k0) * DH;
  const __bf16* vb = (const __bf16*)p.v + (int64_t)head * p.hstride + (int64_t)(start + k0) * DH;

  // max_k |k|^2 over this workgroup's keys (workgroup reduction through LDS).
  float kn2 = 0.f;
  {
    const float* kn = p.knorm + (int64_t)head * (p.hstride / DH) + start + k0;
    // Eight independent loads in flight per thread and round (one memory latency per round).
    for (int r0 = tid; r0 < nk; r0 += 8 * NT) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = r0 + u * NT < nk ? kn[r0 + u * NT] : 0.f;
#pragma unroll
      for (int u = 0; u < 8; ++u) kn2 = fmaxf(kn2, v[u]);
    }
    kn2 = wave_max(kn2);
    float* red = (float*)smem;
    if (lane == 0) red[wave] = kn2;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < NW; ++w) kn2 = fmaxf(kn2, red[w]);
    __syncthreads();
  }

  int qi[QB];
  u32x4 qr[QB][QKG];
  // PIPE: the offset -m_q as the QK^T MFMA's C operand (16 registers per query block). Otherwise no
  // offset while every bound m_q <= 64 (scores, P and the sums stay far inside the FP32 and bf16
  // ranges), else exp2(s - m_q) with the offset kept once per query.
  f32x16 cneg[PIPE ? QB : 1];
  float mq_[QB];
#pragma unroll
  for (int j = 0; j < QB; ++j) {
    qi[j] = (qtile * NW + wave) * (32 * QB) + 32 * j + i;
    float qn2 = 0.f;
#pragma unroll
    for (int c = 0; c < QKG; ++c) {
      qr[j][c] = qi[j] < n ? *(const u32x4*)(qb + (int64_t)qi[j] * DH + (2 * c + h) * 8)
                           : u32x4{0, 0, 0, 0};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float lo = __uint_as_float(qr[j][c][e] << 16), hi = __uint_as_float(qr[j][c][e] & 0xffff0000u);
        qn2 = fmaf(lo, lo, fmaf(hi, hi, qn2));
      }
    }
    qn2 += other_half(qn2);
    // Scores are sums of DH exact products in FP32: |s - q.k| <= DH * 2^-24 |q| |k|.
    const float mq = sqrtf(qn2 * kn2) * (1.f + 0x1p-12f);
    mq_[j] = mq;
    if constexpr (PIPE) {
#pragma unroll
      for (int r = 0; r < 16; ++r) cneg[j][r] = -mq;
    }
  }

  // Bounded buffer loads: zeros past the last key.
  const int run_bytes = nk * DH * 2;
  const __amdgpu_buffer_rsrc_t krs = __builtin_amdgcn_make_buffer_rsrc((void*)kb, (short)0, run_bytes, kBufferWord3);
  const __amdgpu_buffer_rsrc_t vrs = __builtin_amdgcn_make_buffer_rsrc((void*)vb, (short)0, run_bytes, kBufferWord3);
  auto load = [&](int st, u32x4 (&rk)[PT], u32x4 (&rv)[PT]) {
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      const int c = t * NT + tid;
      const int off = (st * KEYS + c / CH_ROW) * (DH * 2) + (c % CH_ROW) * 16;
      rk[t] = __builtin_amdgcn_raw_buffer_load_b128(krs, off, 0, 0);
      rv[t] = __builtin_amdgcn_raw_buffer_load_b128(vrs, off, 0, 0);
    }
  };
  auto store = [&](int slot, const u32x4 (&rk)[PT], const u32x4 (&rv)[PT]) {
    char* Ks = smem + slot * SLOT;
    char* Vs = Ks + K_BYTES;
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      const int c = t * NT + tid;
      if (NCH % NT != 0 && c >= NCH) break;
      const int r = c / CH_ROW, ch = c % CH_ROW;
      *(u32x4*)(Ks + r * KRS + ch * 16) = rk[t];
      *(u32x4*)(Vs + r * VRS + ch * 16) = rv[t];
    }
  };

  float m_ex[QB];
  f32x16 oacc[QB];
  // Row sums of the packed P, of exactly the bf16 values the PV product uses. d_head 32: per lane
  // with v_dot2 (the two lane halves added at the end). d_head 16: V^T rows 16-31 are idle, and
  // row 16 holds ones, so the PV MFMA itself produces the row sum as O^T row 16 (register 8 of the
  // lanes of half 0, zero in half 1) at no VALU cost.
  [[maybe_unused]] float l_run[QB];
  auto reset_sums = [&]() {
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      oacc[j] = f32x16{};
      if constexpr (DH == 32) l_run[j] = 0.f;
    }
  };
  // The full row sum of this lane's query (block j); every lane must call it (lane exchange).
  auto row_sum = [&](int j) {
    if constexpr (DH == 32)
      return l_run[j] + other_half(l_run[j]);
    else
      return oacc[j][8] + other_half(oacc[j][8]);
  };

  // K fragments of key block b (its stage b / G sits in LDS slot (b / G) % 3).
  auto kread = [&](int b, u32x4 (&ka)[QKG]) {
    const char* Ks = smem + ((b / G) % 3) * SLOT;
#pragma unroll
    for (int c = 0; c < QKG; ++c) ka[c] = *(const u32x4*)(Ks + (32 * (b % G) + i) * KRS + (2 * c + h) * 16);
  };
  // Scores plus C from K fragments.
  auto scores = [&](const u32x4 (&ka)[QKG], f32x16 (&s)[QB], const f32x16 (&c0)[QB]) {
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      s[j] = c0[j];
#pragma unroll
      for (int c = 0; c < QKG; ++c) mma_kg<BF16>(ka[c], qr[j][c], s[j]);
    }
  };
  // Keys at or past nk get -inf (only the last block can hold such keys).
  auto mask = [&](int b, f32x16 (&s)[QB]) {
    const int lim = nk - 32 * b - 4 * h;  // key 32b + 4h + c_r is valid iff c_r < lim
#pragma unroll
    for (int j = 0; j < QB; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if (8 * (r >> 2) + (r & 3) >= lim) s[j][r] = -INFINITY;
  };
  // P = exp2(S'), packed to bf16 and summed into l as packed; O^T += V^T P^T.
  typedef short tr4 __attribute__((ext_vector_type(4)));
  typedef __attribute__((address_space(3))) tr4 lds_tr4;
  const int j16 = i & 15;
  const int vcol = ((DH == 32 ? (i & 16) : 0) + 4 * (j16 & 3)) * 2;  // byte column this lane addresses
  float msh[QB];  // the per-query shift of the exponents when SHIFT (PIPE false)
  auto consume = [&](int slot, int bb, const f32x16 (&s)[QB], auto shift_tag) {
    constexpr bool SHIFT = decltype(shift_tag)::value;
    const char* Vs = smem + slot * SLOT + K_BYTES;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      // Keys 16c + 4h + (0..3) and 16c + 8 + 4h + (0..3) of the block, the order of P^T's registers.
      const char* vp = Vs + (32 * bb + 16 * c + 4 * h + (j16 >> 2)) * VRS + vcol;
      const tr4 v0 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_tr4*)vp);
      const tr4 v1 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_tr4*)(vp + 8 * VRS));
      const u32x2 w0 = __builtin_bit_cast(u32x2, v0), w1 = __builtin_bit_cast(u32x2, v1);
      u32x4 va = u32x4{w0[0], w0[1], w1[0], w1[1]};
      if (DH < 32 && i >= DH)
        va = i == DH ? u32x4{0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u} : u32x4{0, 0, 0, 0};
#pragma unroll
      for (int j = 0; j < QB; ++j) {
        u32x4 pb;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const float e0 = __builtin_amdgcn_exp2f(SHIFT ? s[j][8 * c + 4 * q + 0] - msh[j] : s[j][8 * c + 4 * q + 0]);
          const float e1 = __builtin_amdgcn_exp2f(SHIFT ? s[j][8 * c + 4 * q + 1] - msh[j] : s[j][8 * c + 4 * q + 1]);
          const float e2 = __builtin_amdgcn_exp2f(SHIFT ? s[j][8 * c + 4 * q + 2] - msh[j] : s[j][8 * c + 4 * q + 2]);
          const float e3 = __builtin_amdgcn_exp2f(SHIFT ? s[j][8 * c + 4 * q + 3] - msh[j] : s[j][8 * c + 4 * q + 3]);
          const u32x2 pk = pack_bf16x4(e0, e1, e2, e3);
          if constexpr (DH == 32) l_run[j] = add_bf16x4(e0, e1, e2, e3, l_run[j]);
          pb[2 * q] = pk[0];
          pb[2 * q + 1] = pk[1];
        }
        mma_kg<BF16>(va, pb, oacc[j]);
      }
    }
  };
  // Exact-maximum pass: running row maxima of the raw scores.
  auto take_max = [&](const f32x16 (&s)[QB]) {
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      float a = fmaxf(fmaxf(s[j][0], s[j][1]), s[j][2]), b = fmaxf(fmaxf(s[j][3], s[j][4]), s[j][5]);
      a = fmaxf(fmaxf(a, s[j][6]), s[j][7]);
      b = fmaxf(fmaxf(b, s[j][8]), s[j][9]);
      a = fmaxf(fmaxf(a, s[j][10]), s[j][11]);
      b = fmaxf(fmaxf(b, s[j][12]), s[j][13]);
      a = fmaxf(fmaxf(a, s[j][14]), s[j][15]);
      m_ex[j] = fmaxf(m_ex[j], fmaxf(a, b));
    }
  };

  const int nblk = (nk + 31) >> 5;
  const int nst = (nblk + G - 1) / G;
  // One sweep over the keys through the LDS stages; MAXPASS: maxima only.
  auto sweep = [&](auto maxpass_tag, const f32x16 (&c0)[QB], auto shift_tag) {
    constexpr bool MAXPASS = decltype(maxpass_tag)::value;
    {
      u32x4 rk0[PT], rv0[PT], rk1[PT], rv1[PT];
      if (nst > 0) load(0, rk0, rv0);
      if (nst > 1) load(1, rk1, rv1);
      if (nst > 0) store(0, rk0, rv0);
      if (nst > 1) store(1, rk1, rv1);
    }
    __syncthreads();
    u32x4 rk[PT], rv[PT];
    if (nst > 2) load(2, rk, rv);

    f32x16 sa[QB], sb[QB];
    u32x4 kn[QKG];  // K fragments of the next block to score, read a step ahead
    if (PIPE && nblk > 0) {
      kread(0, kn);
      scores(kn, sa, c0);
      if (nblk == 1 && (nk & 31)) mask(0, sa);
    }
    if (PIPE && nblk > 1) kread(1, kn);
    // Block b of stage st (position bb) is in `cur`; the look-ahead product fills `nxt` from the
    // K fragments read during the previous step, and the fragments of block b + 2 (in stage st or
    // st + 1, both resident) are read for the next one. Past the last block both repeat the last
    // block (unused results; no branch, so the fragment registers rotate without copies).
    auto step = [&](int st, int slot, int bb, f32x16 (&cur)[QB], f32x16 (&nxt)[QB]) {
      const int b = st * G + bb;
      {
        u32x4 ka[QKG];
#pragma unroll
        for (int c = 0; c < QKG; ++c) ka[c] = kn[c];
        kread(min(b + 2, nblk - 1), kn);
        scores(ka, nxt, c0);
        if (b + 2 == nblk && (nk & 31)) mask(b + 1, nxt);
      }
      if constexpr (MAXPASS)
        take_max(cur);
      else
        consume(slot, bb, cur, shift_tag);
    };
    // Without the look-ahead (PIPE false): block b is scored and consumed in the same step, with one
    // score set fewer in registers (more waves per SIMD hide the MFMA latency instead).
    auto step_np = [&](int st, int slot, int bb) {
      const int b = st * G + bb;
      u32x4 ka[QKG];
      kread(b, ka);
      scores(ka, sa, c0);
      if (b + 1 == nblk && (nk & 31)) mask(b, sa);
      if constexpr (MAXPASS)
        take_max(sa);
      else
        consume(slot, bb, sa, shift_tag);
    };
    int slot = 0;
    for (int st = 0; st < nst; ++st) {
#pragma unroll
      for (int bb = 0; bb < G; bb += 2) {
        const int b = st * G + bb;
        if constexpr (PIPE) {
          if (b < nblk) step(st, slot, bb, sa, sb);
          if (b + 1 < nblk) step(st, slot, bb + 1, sb, sa);
        } else {
          if (b < nblk) step_np(st, slot, bb);
          if (b + 1 < nblk) step_np(st, slot, bb + 1);
        }
      }
      if (st + 2 < nst) store(slot == 0 ? 2 : slot - 1, rk, rv);
      __syncthreads();
      if (st + 3 < nst) load(st + 3, rk, rv);
      slot = slot == 2 ? 0 : slot + 1;
    }
  };

  reset_sums();
  // The exponent offset of each query's P: -cneg (PIPE), else msh once shifted, 0 before.
  bool shifted = false;
  f32x16 zero[QB];
#pragma unroll
  for (int j = 0; j < QB; ++j) zero[j] = f32x16{};
  if constexpr (PIPE) {
    sweep(std::false_type{}, cneg, std::false_type{});
  } else {
    bool big = false;
#pragma unroll
    for (int j = 0; j < QB; ++j) big = big || (qi[j] < n && !(mq_[j] <= 64.f));
    if (__syncthreads_or(big)) {
      shifted = true;
#pragma unroll
      for (int j = 0; j < QB; ++j) msh[j] = mq_[j];
      sweep(std::false_type{}, zero, std::true_type{});
    } else {
      sweep(std::false_type{}, zero, std::false_type{});
    }
  }

  // Fallback when a bound was too loose: l >= 2^-(bound - max) and that fell below 2^-96.
  bool loose = false;
#pragma unroll
  for (int j = 0; j < QB; ++j) {
    const float l_tot = row_sum(j);
    loose = loose || (qi[j] < n && nk > 0 && !(l_tot >= 0x1p-96f) && l_tot == l_tot);
  }
  if (__syncthreads_or(loose)) {
#pragma unroll
    for (int j = 0; j < QB; ++j) m_ex[j] = -INFINITY;
    sweep(std::true_type{}, zero, std::false_type{});
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      const float mx = fmaxf(m_ex[j], other_half(m_ex[j]));
      if constexpr (PIPE) {
#pragma unroll
        for (int r = 0; r < 16; ++r) cneg[j][r] = -mx;
      } else {
        msh[j] = mx;
      }
    }
    reset_sums();
    shifted = true;
    if constexpr (PIPE)
      sweep(std::false_type{}, cneg, std::false_type{});
    else
      sweep(std::false_type{}, zero, std::true_type{});
  }

  // Key split: the unnormalised O^T, with l and the offset (l = 0 for a split without keys).
  if (p.ksplit > 1) {
    const int nh = p.d / DH;
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      const float l_tot = row_sum(j);
      if (qi[j] < n) {
        const int64_t prow = (int64_t)split * p.rows + start + qi[j];
        float* po = p.part_o + prow * p.d + head * DH + 4 * h;
#pragma unroll
        for (int c = 0; c < DH / 8; ++c)
          *(f32x4*)(po + 8 * c) = f32x4{oacc[j][4 * c], oacc[j][4 * c + 1], oacc[j][4 * c + 2], oacc[j][4 * c + 3]};
        const float moff = PIPE ? -cneg[j][0] : shifted ? msh[j] : 0.f;
        // (the lane's half from its lane id, recomputed here rather than kept through the loop)
        if (__lane_id() < 32) *(f32x2*)(p.part_ml + (prow * nh + head) * 2) = f32x2{moff, l_tot};
      }
    }
    return;
  }

  // O = O^T / l. Lane l holds dh = 8c + 4*(l/32) + (0..3) of query l%32 in registers 4c..4c+3.
#pragma unroll
  for (int j = 0; j < QB; ++j) {
    const float l_tot = row_sum(j);
    if (qi[j] < n) {
      const float inv = 1.0f / l_tot;
      __bf16* orow = (__bf16*)p.o + (int64_t)(start + qi[j]) * p.d + head * DH;
#pragma unroll
      for (int c = 0; c < DH / 8; ++c)
        *(u32x2*)(orow + 8 * c + 4 * h) = pack_bf16x4(oacc[j][4 * c] * inv, oacc[j][4 * c + 1] * inv,
                                                     oacc[j][4 * c + 2] * inv, oacc[j][4 * c + 3] * inv);
    }
  }
}

// Combination of the key-split partial results of one work item (event, head, query tile) per
// workgroup: with M the largest offset among the splits that saw keys, O = sum_s 2^(m_s - M) O_s /
// sum_s 2^(m_s - M) l_s (splits in order), rounded to bf16. One thread per 8 values of a query;
// all of a thread's loads are issued before any result is used.
template <int DH, int S>
__global__ __launch_bounds__(256) void attn_combine_kernel(const AttnArgs p) {
  const int n_it = min(*p.n_items, p.cap_items);
  if ((int)blockIdx.x >= n_it) return;
  const int ev = p.items[2 * blockIdx.x], code = p.items[2 * blockIdx.x + 1];
  const int head = code & 255, qtile = code >> 8;
  const int start = p.ev_start[ev], n = p.ev_n[ev];
  const int nh = p.d / DH;
  constexpr int CH = DH / 8;
  for (int t = threadIdx.x; t < p.q_tile * CH; t += 256) {
    const int qi = qtile * p.q_tile + t / CH, c = t % CH;
    if (qi >= n) continue;
    const int64_t row = start + qi;
    f32x2 ml[S];
    f32x4 oa[S], ob[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int64_t prow = (int64_t)s * p.rows + row;
      ml[s] = *(const f32x2*)(p.part_ml + (prow * nh + head) * 2);
      const float* po = p.part_o + prow * p.d + head * DH + 8 * c;
      oa[s] = *(const f32x4*)po;
      ob[s] = *(const f32x4*)(po + 4);
    }
    float mmax = -INFINITY;
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (ml[s][1] > 0.f) mmax = fmaxf(mmax, ml[s][0]);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float den = 0.f;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      // Splits without keys (l = 0) weigh nothing; their O values are not read into the sums.
      const bool live = ml[s][1] > 0.f;
      const float w = live ? __builtin_amdgcn_exp2f(ml[s][0] - mmax) : 0.f;
      den = fmaf(w, ml[s][1], den);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc[e] = live ? fmaf(w, oa[s][e], acc[e]) : acc[e];
        acc[4 + e] = live ? fmaf(w, ob[s][e], acc[4 + e]) : acc[4 + e];
      }
    }
    const float inv = 1.0f / den;
    const u32x2 lo = pack_bf16x4(acc[0] * inv, acc[1] * inv, acc[2] * inv, acc[3] * inv);
    const u32x2 hi = pack_bf16x4(acc[4] * inv, acc[5] * inv, acc[6] * inv, acc[7] * inv);
    *(u32x4*)((__bf16*)p.o + row * p.d + head * DH + 8 * c) = u32x4{lo[0], lo[1], hi[0], hi[1]};
  }
}

// Squared key norms |k|^2 per (head, row) of a [H][rows][dh] bf16 K, read by the BF16 attention
// kernel for its score bound. One thread per (head, row).
template <int DH>
__global__ __launch_bounds__(256) void keynorm_kernel(const __bf16* k, float* out, int64_t total) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= total) return;
  const u32x4* row = (const u32x4*)(k + t * DH);
  float acc = 0.f;
#pragma unroll
  for (int c = 0; c < DH / 8; ++c) {
    const u32x4 v = row[c];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float lo = __uint_as_float(v[e] << 16), hi = __uint_as_float(v[e] & 0xffff0000u);
      acc = fmaf(lo, lo, fmaf(hi, hi, acc));
    }
  }
  out[t] = acc;
}

namespace {

constexpr AttnTile kTiles[] = {
    // classic kernel (KT keys per LDS tile, two LDS buffers)
    {4, 64, 1, 0},
    {2, 64, 1, 0},
    {4, 32, 1, 0},
    {1, 64, 1, 0},
    {2, 64, 2, 0},
    {4, 64, 2, 0},
    // BF16 bound-offset kernel (stages of KT keys, three LDS slots); FP32 runs the two-buffer
    // kernel of the same shape.
    {4, 64, 1, 1},
    {4, 64, 2, 1},
    {4, 128, 1, 1},
    {2, 64, 1, 1},
    {8, 64, 1, 1},
    {4, 64, 1, 1},  // as 6, registers capped for 4 waves per SIMD
    {2, 64, 2, 1},
    {4, 128, 2, 1},
    // the same without the look-ahead product (kind 2), registers capped for 3 or 4 waves per SIMD
    {4, 64, 2, 2},
    {4, 128, 2, 2},
    {4, 64, 1, 2},
};

template <class T, int DH, int NW, int KT, int QB>
hipError_t launch_t(const AttnArgs& p, hipStream_t s) {
  if (p.cap_items <= 0) return hipSuccess;
  hipLaunchKernelGGL((attn_kernel<T, DH, NW, KT, QB>), dim3(p.cap_items), dim3(NW * 64), 0, s, p);
  return hipGetLastError();
}

template <class T, int DH, int NW, int KT, int QB, int OCC = 1, bool PIPE = true>
hipError_t launch_b(const AttnArgs& p, hipStream_t s) {
  if constexpr (!std::is_same_v<T, BF16>) {
    return launch_t<T, DH, NW, KT, QB>(p, s);
  } else {
    if (p.cap_items <= 0) return hipSuccess;
    if (p.knorm == nullptr || (p.ksplit != 1 && p.ksplit != 2 && p.ksplit != 4 && p.ksplit != 8) ||
        (p.ksplit > 1 && (p.part_o == nullptr || p.part_ml == nullptr)))
      return hipErrorInvalidValue;
    hipLaunchKernelGGL((attn_bf16_kernel<DH, NW, KT / 32, QB, OCC, PIPE>), dim3(p.cap_items * p.ksplit),
                       dim3(NW * 64), 0, s, p);
    return hipGetLastError();
  }
}

template <class T, int DH>
hipError_t launch_dh(int tile, const AttnArgs& p, hipStream_t s) {
  switch (tile) {
    case 0: return launch_t<T, DH, 4, 64, 1>(p, s);
    case 1: return launch_t<T, DH, 2, 64, 1>(p, s);
    case 2: return launch_t<T, DH, 4, 32, 1>(p, s);
    case 3: return launch_t<T, DH, 1, 64, 1>(p, s);
    case 4: return launch_t<T, DH, 2, 64, 2>(p, s);
    case 5: return launch_t<T, DH, 4, 64, 2>(p, s);
    case 6: return launch_b<T, DH, 4, 64, 1>(p, s);
    case 7: return launch_b<T, DH, 4, 64, 2>(p, s);
    case 8: return launch_b<T, DH, 4, 128, 1>(p, s);
    case 9: return launch_b<T, DH, 2, 64, 1>(p, s);
    case 10: return launch_b<T, DH, 8, 64, 1>(p, s);
    case 11: return launch_b<T, DH, 4, 64, 1, 4>(p, s);
    case 12: return launch_b<T, DH, 2, 64, 2>(p, s);
    case 13: return launch_b<T, DH, 4, 128, 2>(p, s);
    case 14: return launch_b<T, DH, 4, 64, 2, 3, false>(p, s);
    case 15: return launch_b<T, DH, 4, 128, 2, 3, false>(p, s);
    case 16: return launch_b<T, DH, 4, 64, 1, 4, false>(p, s);
    default: return hipErrorInvalidValue;
  }
}

template <class T>
hipError_t launch_prec(int tile, const AttnArgs& p, hipStream_t s) {
  if (p.dh == 32) return launch_dh<T, 32>(tile, p, s);
  if (p.dh == 16) return launch_dh<T, 16>(tile, p, s);
  return hipErrorInvalidValue;
}

}  // namespace

int attn_num_tiles() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }
AttnTile attn_tile(int id) { return kTiles[id]; }

hipError_t launch_keynorm(const void* k, float* out, int64_t total, int dh, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  const int64_t blocks = (total + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (dh == 32)
    hipLaunchKernelGGL(keynorm_kernel<32>, dim3((unsigned)blocks), dim3(256), 0, s, (const __bf16*)k, out, total);
  else if (dh == 16)
    hipLaunchKernelGGL(keynorm_kernel<16>, dim3((unsigned)blocks), dim3(256), 0, s, (const __bf16*)k, out, total);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_attn_combine(const AttnArgs& p, hipStream_t s) {
  if (p.cap_items <= 0) return hipSuccess;
  if ((p.ksplit != 2 && p.ksplit != 4 && p.ksplit != 8) || !p.part_o || !p.part_ml || p.q_tile <= 0)
    return hipErrorInvalidValue;
  if (p.dh != 32 && p.dh != 16) return hipErrorInvalidValue;
  auto go = [&](auto dh_tag) {
    constexpr int DH = decltype(dh_tag)::value;
    switch (p.ksplit) {
      case 2: hipLaunchKernelGGL((attn_combine_kernel<DH, 2>), dim3(p.cap_items), dim3(256), 0, s, p); break;
      case 4: hipLaunchKernelGGL((attn_combine_kernel<DH, 4>), dim3(p.cap_items), dim3(256), 0, s, p); break;
      default: hipLaunchKernelGGL((attn_combine_kernel<DH, 8>), dim3(p.cap_items), dim3(256), 0, s, p); break;
    }
  };
  if (p.dh == 32)
    go(std::integral_constant<int, 32>{});
  else
    go(std::integral_constant<int, 16>{});
  return hipGetLastError();
}

hipError_t launch_attention(Prec prec, int tile, const AttnArgs& p, hipStream_t s) {
  if (prec == P_F32) return launch_prec<F32>(tile, p, s);
  if (prec == P_BF16) return launch_prec<BF16>(tile, p, s);
  return hipErrorInvalidValue;
}

}  // namespace mlpf
