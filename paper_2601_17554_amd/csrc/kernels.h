// Host-side launch interfaces of the libmlpf kernels (internal; the public ABI is mlpf.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlpf {

enum Prec { P_F32 = 0, P_BF16 = 1, P_FP8 = 2 };

// How the GEMM's A operand is produced while it is staged into LDS.
enum ALoad {
  A_PLAIN = 0,   // A already holds the operand type (row stride lda, K % 16 bytes == 0)
  A_F32 = 1,     // A is FP32, converted to the operand type
  A_SCALAR = 2,  // A is FP32 with any K and row stride (element loads, zero beyond K)
};

// What the GEMM does with acc = A W (+ bias) for each output element.
enum Epi {
  E_BIAS = 0,    // out_f32[row][col] = acc + bias
  E_RESID = 1,   // out_f32[row][col] += acc + bias           (residual update, in place)
  E_GELU = 2,    // out_T[row][col] = GELU(acc + bias)
  E_QKV = 3,     // Q (scaled), K, V written head-major [head][row][d_head] in the operand type
  E_BIAS_B = 4,  // out_bf16[row][col] = acc + bias            (bf16 residual stream)
  E_RESID_B = 5, // out_bf16[row][col] = bf16(out + acc + bias), the sum taken in FP32
  E_HEADS = 6,   // first head layer (GELU, bf16) and, per 256-wide head tile, its second-layer
                 // outputs: hout[row][cols of head] = hidden . W2[:, cols] (biases added later)
};

struct GemmArgs {
  const void* a = nullptr;  // A [M][lda]
  int lda = 0;
  int M = 0, N = 0, K = 0;  // logical sizes; K is the reduction length
  int Kp = 0;               // row length of wt (K rounded up to the k-tile)
  const void* wt = nullptr; // W^T [N][Kp] in the operand type
  const float* bias = nullptr;
  const int32_t* m_dev = nullptr;  // optional device count of live rows (rows beyond it are skipped)
  void* out = nullptr;
  int ldo = 0;
  float acc_scale = 1.f;   // multiplies A W before the bias (FP8 dequantisation s_a * s_w)
  float out_scale = 1.f;   // E_GELU into FP8: multiplies GELU(...) before rounding (1 / s_out)
  float* amax = nullptr;   // E_GELU: optional running max |GELU(...)| (calibration; atomic max)
  int relu = 0;            // E_GELU, E_HEADS: ReLU instead of GELU
  // E_QKV
  void* q = nullptr;
  void* k = nullptr;
  void* v = nullptr;
  int64_t hstride = 0;  // elements between heads in q/k/v (= rows capacity * d_head)
  int d = 0, dh = 0;
  float q_scale = 1.f;
  float* knorm = nullptr;  // bf16 E_QKV: also write |k|^2 per (head, row), [H][hstride / dh]
  // E_HEADS
  const float* w2 = nullptr;  // [256][11]
  float* hout = nullptr;      // [M][11]
  int head0 = 0;              // head index of the first 256 columns
  int heads6 = 0;             // six heads (binary 1, pid 5, pT 1, eta 1, phi 2, E 1) instead of five
};

// Tile shapes available to the GEMM (index = tile id). Each entry: BM, BN, BK(bytes-agnostic
// elements), waves along M, waves along N.
struct GemmTile {
  int bm, bn, wm, wn;
  int bkb;      // bytes of each operand row per k-tile
  int persist;  // 1: persistent workgroups looping over tiles; 2: k-tiles by direct-to-LDS loads
                // through three LDS stages (plain A operands)
};
int gemm_num_tiles();
GemmTile gemm_tile(int id);
hipError_t launch_gemm(Prec prec, ALoad aload, Epi epi, int tile, const GemmArgs& args,
                       hipStream_t stream);

// Fused BF16 FFN block: h[M][d_model] += GELU(y W1 + b1) W2 + b2 with the weights pre-tiled by
// ffn_pack (W1 and W2 chunks of 64 hidden units as their LDS images).
struct FfnArgs {
  const void* y = nullptr;      // bf16 [M][d_model]: LN2(h), or h itself when ln_in_g is set
  const float* ln_in_g = nullptr;  // optional: y = LayerNorm(rows of y) computed in the kernel
  const float* ln_in_b = nullptr;
  float ln_in_eps = 1e-5f;
  int M = 0;
  const int32_t* m_dev = nullptr;
  int d_model = 0, d_ff = 0;
  const void* w1p = nullptr;    // ffn_pack layout
  const float* b1 = nullptr;
  const void* w2p = nullptr;
  const float* b2 = nullptr;
  int relu = 0;                 // ReLU instead of GELU
  // FP8 form (launch_ffn_fp8): y = E4M3(LN2(h) * fp8_in_scale); U = E4M3(act(acc1 * acc_scale + b1)
  // * out_scale); h += acc2 * acc_scale2 + b2 (the per-tensor scales 1/s_a1, s_a1 s_w1, 1/s_a2,
  // s_a2 s_w2).
  float fp8_in_scale = 1.f, acc_scale = 1.f, out_scale = 1.f, acc_scale2 = 1.f;
  void* h = nullptr;            // bf16 [M][d_model], updated in place (sum taken in FP32)
  // Optional: the next block's LN1 of the updated h, written as bf16 [M][d_model] (the operand of
  // the next QKV projection), bitwise equal to the LayerNorm kernel's output.
  void* y_next = nullptr;
  const float* ln_g = nullptr;
  const float* ln_b = nullptr;
  float ln_eps = 1e-5f;
  // Variant 5: the hidden units in `split` equal parts (a divisor of d_ff / 64), one workgroup per
  // (row tile, part) writing its FP32 partial product to part [split][M][d_model]; a reduction
  // kernel then updates h (and writes y_next).
  int split = 1;
  float* part = nullptr;
};
int ffn_fused_supported(int d_model, int d_ff);
// Bytes of the packed W1 (which = 1) or W2 (which = 2) image.
size_t ffn_pack_bytes(int d_model, int d_ff, int which);
// Packs W1^T [d_ff][d_model] and W2^T [d_model][d_ff] (bf16 bits) into the chunked images.
void ffn_pack(const uint16_t* w1t, const uint16_t* w2t, int d_model, int d_ff, uint16_t* w1p,
              uint16_t* w2p);
// variant 1: 128 rows x 8 waves, double-buffered weights; 2: 64 rows x 4 waves, single-buffered.
hipError_t launch_ffn_fused(const FfnArgs& args, int variant, hipStream_t stream);
// The FP8-E4M3 form (persistent, 128 rows x 8 waves, LN2 always computed from h: args.y = h and
// ln_in_g set), weights packed by ffn_fp8_pack: W1^T [d_ff][d_model] and W2^T [d_model][d_ff] E4M3
// bytes into chunk images of 64 hidden units.
size_t ffn_fp8_pack_bytes(int d_model, int d_ff, int which);
void ffn_fp8_pack(const uint8_t* w1t, const uint8_t* w2t, int d_model, int d_ff, uint8_t* w1p,
                  uint8_t* w2p);
hipError_t launch_ffn_fp8(const FfnArgs& args, hipStream_t stream);

// Attention over a device work list (see worklist).
struct AttnArgs {
  const void* q = nullptr;  // [H][rows_cap][dh], pre-scaled by log2(e)/sqrt(dh)
  const void* k = nullptr;
  const void* v = nullptr;
  void* o = nullptr;        // [rows][d]
  int64_t hstride = 0;
  int d = 0, dh = 0;
  const int32_t* items = nullptr;    // [cap][2]: event, (q_tile << 8) | head
  const int32_t* n_items = nullptr;  // device count
  const int32_t* ev_start = nullptr;
  const int32_t* ev_n = nullptr;
  const float* knorm = nullptr;      // BF16 kernel: [H][rows_cap] squared key norms
  int cap_items = 0;
  // Key split (BF16 bound-offset kernel): ksplit > 1 runs every work item as ksplit workgroups,
  // each over one contiguous range of the event's keys, writing for each of its queries the
  // unnormalised O (part_o [ksplit][rows][d], FP32), and the exponent offset and row sum
  // (part_ml [ksplit][rows][H], (m, l)); launch_attn_combine then forms O. Grid: ksplit x
  // cap_items workgroups, split-major.
  int ksplit = 1;
  int rows = 0;       // rows of the partial buffers (the batch's total rows)
  int q_tile = 0;     // queries per work item
  float* part_o = nullptr;
  float* part_ml = nullptr;
};
struct AttnTile {
  int waves;  // waves per workgroup
  int kt;     // keys per LDS tile
  int qb;     // 32-query blocks per wave; queries per work item = 32 * waves * qb
  int kind;   // 0: two-buffer online-softmax kernel; 1: BF16 bound-offset kernel (needs knorm);
              // 2: the bound-offset kernel without the look-ahead product
};
int attn_num_tiles();
AttnTile attn_tile(int id);
hipError_t launch_attention(Prec prec, int tile, const AttnArgs& args, hipStream_t stream);
// O of every work item's valid queries from the ksplit partial results (bf16 output).
hipError_t launch_attn_combine(const AttnArgs& args, hipStream_t stream);
// knorm[t] = |k_t|^2 for the total = H * rows_cap rows of a bf16 [H][rows_cap][dh] K.
hipError_t launch_keynorm(const void* k, float* knorm, int64_t total, int dh, hipStream_t stream);

// Sanitises the batch description and builds the attention work list (one workgroup).
struct WorklistArgs {
  const int32_t* row_start = nullptr;
  const int32_t* n_valid = nullptr;
  int n_events = 0, total_rows = 0, max_seqlen = 0;
  int q_tile = 32, n_heads = 1, cap_items = 0;
  int32_t* ev_start = nullptr;
  int32_t* ev_n = nullptr;
  int32_t* items = nullptr;
  int32_t* n_items = nullptr;
  int32_t* n_rows = nullptr;
};
hipError_t launch_worklist(const WorklistArgs& args, hipStream_t stream);

// Second layer of the output heads, class rule and optional decode.
struct Heads2Args {
  const void* uh = nullptr;   // [rows][nh d] hidden activations (operand type), nh = 5 or 6
  int d = 0, rows = 0;
  const int32_t* m_dev = nullptr;
  const float* w2 = nullptr;  // [d][11]: columns cls0..5 (or binary, pid1..5), pt, eta, sin, cos, e
  const float* b2 = nullptr;  // [11]
  float* logits = nullptr;
  float* reg = nullptr;
  int32_t* cls = nullptr;
  const float* prim = nullptr;
  float* decoded = nullptr;
  int binary = 0;  // class rule: 0 argmax of six (class 0 = none), 1 binary logit > 0 then PID argmax
  int heads6 = 0;  // uh holds six heads' hidden layers (binary, pid, pT, eta, phi, E) instead of five
};
hipError_t launch_heads2(Prec prec, const Heads2Args& args, hipStream_t stream);
// From the E_HEADS partial outputs (uh = hout [rows][11] FP32): adds b2, writes logits, reg,
// cls (argmax) and the optional decode.
hipError_t launch_heads_finish(const Heads2Args& args, hipStream_t stream);

// LayerNorm of FP32 or bf16 rows [rows][d] into y [rows][d] of the operand type.
struct LayerNormArgs {
  const void* x = nullptr;
  int x_bf16 = 0;          // 1: x holds bf16 values
  void* y = nullptr;
  int rows = 0, d = 0;
  const int32_t* m_dev = nullptr;
  const float* gamma = nullptr;
  const float* beta = nullptr;
  float eps = 1e-5f;
  float out_scale = 1.f;   // FP8 output: multiplies the normalised value before rounding
  float* amax = nullptr;   // optional running max |LN(x)| (calibration; atomic max)
};
hipError_t launch_layernorm(Prec prec, const LayerNormArgs& args, hipStream_t stream);

// dst[i] = src[i] * scale for n elements of the operand type.
hipError_t launch_scale(Prec prec, void* dst, const void* src, int64_t n, float scale,
                        hipStream_t stream);

// Rows r < min(rows, *m_dev) whose x[r][0] is not above 0.5 get row r of alt (row_bytes each, a
// multiple of 16): the non-track rows of a per-type embedding.
hipError_t launch_select_rows(void* h, const void* alt, const float* x, int n_features, int rows,
                              const int32_t* m_dev, int row_bytes, hipStream_t stream);

// Copies n 4-byte words (duplicates the embedding into the second stack of PARALLEL2).
hipError_t launch_copy_f32(float* dst, const float* src, int64_t n, hipStream_t stream);

}  // namespace mlpf
