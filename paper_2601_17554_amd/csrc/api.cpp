// libmlpf C ABI: argument validation, weight packing, workspace layout and the launch sequence
// of the MLPF forward pass (declared and documented in include/mlpf.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mlpf.h"
#include "candidates.h"
#include "kernels.h"

using namespace mlpf;

namespace {

thread_local std::string g_last_error;

mlpf_status_t fail(mlpf_status_t st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

mlpf_status_t hip_fail(hipError_t e, const char* what) {
  return fail(MLPF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                   \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
  const uint32_t rounding = ((u >> 16) & 1u) + 0x7fffu;
  return (uint16_t)((u + rounding) >> 16);
}

// Padded reduction length of the embedding's first product (F <= 32 features, k-tiles <= 64).
constexpr int kEmbedKp = 64;
constexpr int kHeadsTile = 13;  // the 64 x 256 GEMM tile (whole heads per column tile)

// Output heads: five (cls 6, pT' 1, eta 1, phi 2, E' 1), or six with the paper's separate binary
// and particle-type heads (binary 1, pid 5, then the same four). Their second layers give 11
// outputs in both cases: six classification logits, then pT', eta, sin phi, cos phi, E'.
int n_out_heads(const mlpf_config_t& c) { return c.binary_head ? 6 : 5; }
int n_cls_heads(const mlpf_config_t& c) { return c.binary_head ? 2 : 1; }
const int* head_widths(const mlpf_config_t& c) {
  static const int five[5] = {6, 1, 1, 2, 1};
  static const int six[6] = {1, 5, 1, 1, 2, 1};
  return c.binary_head ? six : five;
}

struct Layer {
  size_t ln1g, ln1b, wqkv, bqkv, wo, bo, ln2g, ln2b, w1, b1, w2, b2;
  size_t w1p = 0, w2p = 0;  // fused-FFN weight images (ffn_pack), when ffn_fused

  // FP8 FFN: per-tensor weight scales and activation scales (FFN1 input, FFN2 input).
  float s_w1 = 1.f, s_w2 = 1.f, s_a1 = 1.f, s_a2 = 1.f;
};

// Byte offsets of every packed tensor inside the device weight buffer.
struct WeightPlan {
  size_t e_w1, e_b1, e_w2, e_b2;
  size_t c_w1 = 0, c_b1 = 0, c_w2 = 0, c_b2 = 0;  // second (non-track) embedding, embed_per_type
  bool ffn_fused = false;  // a fused FFN kernel applies (BF16, or FP8; its weight images are packed)
  bool heads_fused = false;  // the head GEMM can take the second head layer into its epilogue
  std::vector<Layer> layers;
  size_t h_w1, h_b1, h_w2, h_b2;
  size_t total;
};

int elem_bytes(mlpf_precision_t p) { return p == MLPF_FP32 ? 4 : 2; }
int ffn_elem_bytes(mlpf_precision_t p) { return p == MLPF_BF16_FP8FFN ? 1 : elem_bytes(p); }

// OCP FP8 E4M3 (bias 7, max 448, 0x7f = NaN): value of a non-negative code.
double e4m3_value(int c) {
  const int e = c >> 3, m = c & 7;
  return e == 0 ? (m / 8.0) * std::ldexp(1.0, -6) : (1.0 + m / 8.0) * std::ldexp(1.0, e - 7);
}

// Round to nearest (ties to even code) with saturation at +-448.
uint8_t f32_to_e4m3(float x) {
  if (std::isnan(x)) return 0x7f;
  const uint8_t sign = std::signbit(x) ? 0x80 : 0;
  const double a = std::fabs((double)x);
  if (a >= 448.0) return sign | 0x7e;
  int lo = 0, hi = 0x7e;
  while (lo < hi) {  // largest code with value <= a
    const int mid = (lo + hi + 1) / 2;
    if (e4m3_value(mid) <= a) lo = mid;
    else hi = mid - 1;
  }
  const double d0 = a - e4m3_value(lo), d1 = e4m3_value(lo + 1) - a;
  const int c = d0 < d1 ? lo : d0 > d1 ? lo + 1 : ((lo & 1) ? lo + 1 : lo);
  return sign | (uint8_t)c;
}

// Per-tensor E4M3 scale: the largest magnitude maps to 448, the largest finite E4M3 value.
float fp8_scale(float amax) { return amax > 0.f ? amax / 448.0f : 1.0f; }

WeightPlan plan_weights(const mlpf_config_t& c, mlpf_precision_t prec) {
  const size_t d = c.d_model, ff = c.d_ff, eb = elem_bytes(prec), fb = ffn_elem_bytes(prec);
  WeightPlan w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  w.e_w1 = take(d * kEmbedKp * eb);
  w.e_b1 = take(d * 4);
  w.e_w2 = take(d * d * eb);
  w.e_b2 = take(d * 4);
  if (c.embed_per_type) {
    w.c_w1 = take(d * kEmbedKp * eb);
    w.c_b1 = take(d * 4);
    w.c_w2 = take(d * d * eb);
    w.c_b2 = take(d * 4);
  }
  w.layers.resize(c.n_layers);
  w.ffn_fused = prec != MLPF_FP32 && ffn_fused_supported(c.d_model, c.d_ff);
  w.heads_fused = prec != MLPF_FP32 && c.d_model == 256;
  for (auto& L : w.layers) {
    L.ln1g = take(d * 4);
    L.ln1b = take(d * 4);
    L.wqkv = take(3 * d * d * eb);
    L.bqkv = take(3 * d * 4);
    L.wo = take(d * d * eb);
    L.bo = take(d * 4);
    L.ln2g = take(d * 4);
    L.ln2b = take(d * 4);
    L.w1 = take(ff * d * fb);
    L.b1 = take(ff * 4);
    L.w2 = take(d * ff * fb);
    L.b2 = take(d * 4);
    if (w.ffn_fused && prec == MLPF_BF16) {
      L.w1p = take(ffn_pack_bytes(c.d_model, c.d_ff, 1));
      L.w2p = take(ffn_pack_bytes(c.d_model, c.d_ff, 2));
    } else if (w.ffn_fused) {
      L.w1p = take(ffn_fp8_pack_bytes(c.d_model, c.d_ff, 1));
      L.w2p = take(ffn_fp8_pack_bytes(c.d_model, c.d_ff, 2));
    }
  }
  const size_t nh = n_out_heads(c);
  w.h_w1 = take(nh * d * d * eb);
  w.h_b1 = take(nh * d * 4);
  w.h_w2 = take(d * 11 * 4);
  w.h_b2 = take(11 * 4);
  w.total = off;
  return w;
}

size_t master_count(const mlpf_config_t& c) {
  const size_t d = c.d_model, f = c.n_features, ff = c.d_ff;
  size_t n = (c.embed_per_type ? 2 : 1) * (f * d + d + d * d + d);
  n += (size_t)c.n_layers * (2 * d + 3 * d * d + 3 * d + d * d + d + 2 * d + d * ff + ff + ff * d + d);
  n += (size_t)n_out_heads(c) * (d * d + d) + d * 11 + 11;
  return n;
}

mlpf_status_t check_config(const mlpf_config_t* c) {
  if (!c) return fail(MLPF_ERR_INVALID_ARG, "config is NULL");
  if (c->n_features < 1 || c->n_features > 32)
    return fail(MLPF_ERR_UNSUPPORTED, "n_features=%d not in 1..32", c->n_features);
  if (c->d_model < 64 || c->d_model > 1024 || c->d_model % 64)
    return fail(MLPF_ERR_UNSUPPORTED, "d_model=%d must be a multiple of 64 in 64..1024", c->d_model);
  if (c->n_heads < 1 || c->d_model % c->n_heads)
    return fail(MLPF_ERR_INVALID_ARG, "n_heads=%d does not divide d_model", c->n_heads);
  const int dh = c->d_model / c->n_heads;
  if (dh != 16 && dh != 32) return fail(MLPF_ERR_UNSUPPORTED, "d_head=%d must be 16 or 32", dh);
  if (c->n_heads > 255) return fail(MLPF_ERR_UNSUPPORTED, "n_heads > 255");
  if (c->d_ff < 64 || c->d_ff > 4096 || c->d_ff % 64)
    return fail(MLPF_ERR_UNSUPPORTED, "d_ff=%d must be a multiple of 64 in 64..4096", c->d_ff);
  if (c->n_layers < 1 || c->n_layers > 64)
    return fail(MLPF_ERR_UNSUPPORTED, "n_layers=%d not in 1..64", c->n_layers);
  if (c->topology != MLPF_TOPO_SERIAL && c->topology != MLPF_TOPO_PARALLEL2)
    return fail(MLPF_ERR_INVALID_ARG, "unknown topology %d", c->topology);
  if (c->topology == MLPF_TOPO_PARALLEL2 && c->n_layers % 2)
    return fail(MLPF_ERR_INVALID_ARG, "PARALLEL2 needs an even n_layers");
  if (!(c->ln_eps > 0.f) || !std::isfinite(c->ln_eps))
    return fail(MLPF_ERR_INVALID_ARG, "ln_eps must be positive");
  if (c->activation != MLPF_ACT_GELU && c->activation != MLPF_ACT_RELU)
    return fail(MLPF_ERR_INVALID_ARG, "unknown activation %d", c->activation);
  if (c->decision != MLPF_DECIDE_ARGMAX && c->decision != MLPF_DECIDE_BINARY)
    return fail(MLPF_ERR_INVALID_ARG, "unknown decision %d", c->decision);
  if (c->embed_per_type != 0 && c->embed_per_type != 1)
    return fail(MLPF_ERR_INVALID_ARG, "embed_per_type must be 0 or 1");
  if (c->binary_head != 0 && c->binary_head != 1)
    return fail(MLPF_ERR_INVALID_ARG, "binary_head must be 0 or 1");
  return MLPF_OK;
}

}  // namespace

struct mlpf_model_s {
  mlpf_config_t cfg;
  mlpf_precision_t prec;
  Prec kprec;
  int dh;
  int stacks;
  int hbytes;  // bytes per residual-stream element: 4 (MLPF_FP32) or 2 (bf16, the BF16 modes)
  WeightPlan plan;
  const char* base;  // device weight buffer
  // Launch choices (tile ids, -1 = size-based rule), set by mlpf_tune_set.
  int tune[MLPF_OP_COUNT];
  // Optional per-kernel-class timing (mlpf_profiler_*). Event pairs are recorded on the launch
  // stream around every launch of a class while enabled.
  std::mutex prof_mu;
  bool prof_on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events[MLPF_PROF_CLASSES];
  size_t prof_used[MLPF_PROF_CLASSES] = {};
  const void* at(size_t off) const { return base + off; }
  const float* atf(size_t off) const { return (const float*)(base + off); }
};

namespace {

// Workspace layout for a batch of T rows and E events.
struct WsPlan {
  size_t ev_start, ev_n, counters, items, knorm, q, k, v, o, y, u, h, part_o, part_ml, total;
  int cap_items;
  int split_cap;  // most key splits the attention may use (partial buffers for that many)
};

// Key splits of the BF16 attention are for batches too small to fill the chip: at most 8, 4 or 2
// for up to 4096, 8192 or 16384 rows, none beyond (the partial buffers then hold at most 32768
// rows' worth of FP32 outputs).
int attn_split_cap(int64_t T) { return T <= 4096 ? 8 : T <= 8192 ? 4 : T <= 16384 ? 2 : 1; }

WsPlan plan_ws(const mlpf_model_s* m, int64_t T, int64_t E) {
  const mlpf_config_t& c = m->cfg;
  const size_t eb = elem_bytes(m->prec);
  WsPlan w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  // Work items: at most n_heads * sum_e ceil(n_e / 32) <= n_heads * (ceil(T / 32) + E).
  const int64_t cap = (int64_t)c.n_heads * ((T + 31) / 32 + E);
  w.cap_items = (int)std::min<int64_t>(cap, 0x7fffffff);
  w.ev_start = take(E * 4);
  w.ev_n = take(E * 4);
  w.counters = take(16);
  w.items = take((size_t)w.cap_items * 8);
  w.knorm = take((size_t)T * c.n_heads * 4);
  const size_t td = (size_t)T * c.d_model;
  w.q = take(td * eb);
  w.k = take(td * eb);
  w.v = take(td * eb);
  w.o = take(td * eb);
  w.y = take(td * eb);
  const size_t uw = std::max<size_t>((size_t)c.d_ff, (size_t)n_out_heads(c) * c.d_model);
  w.u = take((size_t)T * uw * eb);
  w.h = take((size_t)m->stacks * td * m->hbytes);
  w.split_cap = m->kprec == P_BF16 ? attn_split_cap(T) : 1;
  if (w.split_cap > 1) {
    w.part_o = take((size_t)w.split_cap * td * 4);
    w.part_ml = take((size_t)w.split_cap * T * c.n_heads * 8);
  }
  w.total = off;
  return w;
}

// Size-based default tile: enough workgroups to fill 256 CUs; BF16/FP8 take the 64-byte k-tile
// shapes (more workgroups resident per CU).
int pick_gemm_tile(int M, int N, int kp_bytes, Prec prec) {
  const double wg256 = 256.0;
  const bool narrow = prec != P_F32;
  if ((double)((M + 127) / 128) * ((N + 127) / 128) >= 2 * wg256) return narrow ? 6 : 2;
  if ((double)((M + 127) / 128) * ((N + 63) / 64) >= wg256) return narrow ? 7 : 1;
  return kp_bytes % 128 ? 8 : 0;  // rows of fewer or odd 64-byte k-tiles take the 64-byte shape
}

mlpf_status_t check_layout(const mlpf_batch_t* b);

// The batch and, when given, its attention partitions: each checked on its own, and with host
// mirrors the partitions must tile every event's valid rows, in order, inside the event.
mlpf_status_t check_batch(const mlpf_model_s* m, const mlpf_batch_t* b) {
  (void)m;
  mlpf_status_t st = check_layout(b);
  if (st || !b->attn_parts) return st;
  const mlpf_batch_t* q = b->attn_parts;
  if (q->attn_parts) return fail(MLPF_ERR_INVALID_ARG, "attention partitions cannot have partitions");
  if (q->total_rows != b->total_rows)
    return fail(MLPF_ERR_INVALID_ARG, "attention partitions span %d rows, the batch %d", q->total_rows,
                b->total_rows);
  if ((st = check_layout(q))) return st;
  if (!b->row_start_host) return MLPF_OK;
  if (!q->row_start_host)
    return fail(MLPF_ERR_INVALID_ARG, "the batch has host mirrors, its attention partitions none");
  const int32_t *rs = b->row_start_host, *ps = q->row_start_host;
  int e = 0, pos = 0, end = 0;  // coverage of event e's valid rows reached `pos`
  auto valid_end = [&](int ev) { return rs[ev] + (b->n_valid ? b->n_valid_host[ev] : rs[ev + 1] - rs[ev]); };
  if (b->n_events > 0) {
    pos = rs[0];
    end = valid_end(0);
  }
  for (int p = 0; p < q->n_events; ++p) {
    const int pn = q->n_valid ? q->n_valid_host[p] : ps[p + 1] - ps[p];
    if (pn == 0) continue;
    while (e < b->n_events && pos == end) {  // event e fully covered: on to the next one
      if (++e < b->n_events) {
        pos = rs[e];
        end = valid_end(e);
      }
    }
    if (e >= b->n_events || ps[p] != pos || ps[p] + pn > end)
      return fail(MLPF_ERR_INVALID_ARG, "attention partition %d (rows %d..%d) does not continue the "
                  "valid rows of an event in order", p, ps[p], ps[p] + pn - 1);
    pos += pn;
  }
  while (e < b->n_events && pos == end)
    if (++e < b->n_events) {
      pos = rs[e];
      end = valid_end(e);
    }
  if (e < b->n_events)
    return fail(MLPF_ERR_INVALID_ARG, "valid rows of event %d are in no attention partition", e);
  return MLPF_OK;
}

mlpf_status_t check_layout(const mlpf_batch_t* b) {
  if (!b) return fail(MLPF_ERR_INVALID_ARG, "batch is NULL");
  if (b->n_events < 0 || b->total_rows < 0)
    return fail(MLPF_ERR_INVALID_ARG, "negative n_events or total_rows");
  if (b->max_seqlen < 0) return fail(MLPF_ERR_INVALID_ARG, "negative max_seqlen");
  if (b->max_seqlen > MLPF_MAX_SEQLEN)
    return fail(MLPF_ERR_UNSUPPORTED, "max_seqlen=%d exceeds %d", b->max_seqlen, MLPF_MAX_SEQLEN);
  if (b->n_events > 0 && !b->row_start) return fail(MLPF_ERR_INVALID_ARG, "row_start is NULL");
  // Host mirrors: the documented layout is checked before anything is enqueued.
  const int32_t* rs = b->row_start_host;
  if (!rs) return MLPF_OK;
  if (b->n_valid && !b->n_valid_host)
    return fail(MLPF_ERR_INVALID_ARG, "n_valid_host is needed with row_start_host when n_valid is set");
  if (rs[0] < 0) return fail(MLPF_ERR_INVALID_ARG, "row_start[0]=%d is negative", rs[0]);
  for (int e = 0; e < b->n_events; ++e) {
    if (rs[e + 1] < rs[e])
      return fail(MLPF_ERR_INVALID_ARG, "row_start decreases at event %d (%d > %d)", e, rs[e], rs[e + 1]);
    const int span = rs[e + 1] - rs[e];
    const int nv = b->n_valid ? b->n_valid_host[e] : span;
    if (nv < 0 || nv > span)
      return fail(MLPF_ERR_INVALID_ARG, "n_valid[%d]=%d outside 0..%d (its rows)", e, nv, span);
    if (nv > b->max_seqlen)
      return fail(MLPF_ERR_INVALID_ARG, "event %d has %d valid rows > max_seqlen=%d", e, nv, b->max_seqlen);
  }
  if (rs[b->n_events] > b->total_rows)
    return fail(MLPF_ERR_INVALID_ARG, "row_start[%d]=%d > total_rows=%d", b->n_events, rs[b->n_events],
                b->total_rows);
  return MLPF_OK;
}

// Records a HIP event pair around the launches of one kernel class while profiling is enabled.
struct ProfScope {
  mlpf_model_s* m;
  hipStream_t s;
  hipEvent_t stop = nullptr;
  ProfScope(mlpf_model_s* model, int cls, hipStream_t stream) : m(model), s(stream) {
    if (!m->prof_on) return;
    std::lock_guard<std::mutex> g(m->prof_mu);
    auto& v = m->prof_events[cls];
    size_t& used = m->prof_used[cls];
    if (used == v.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess) return;
      if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
      }
      v.push_back({a, b});
    }
    (void)hipEventRecord(v[used].first, s);
    stop = v[used].second;
    ++used;
  }
  ~ProfScope() {
    if (stop) (void)hipEventRecord(stop, s);
  }
};

struct Ctx {
  mlpf_model_s* m;
  const mlpf_batch_t* b;
  WsPlan w;
  char* ws;
  hipStream_t s;
  const int32_t* n_rows;  // device count of live rows, or NULL
  float* calib = nullptr; // FP8 calibration: [2 L] running amax of the FFN inputs, or NULL
  void* p(size_t off) const { return ws + off; }
};

// Default attention tile: BF16 takes the score-bound kernel, 4 waves x 2 query blocks, no look-ahead
// product, three waves per SIMD.
constexpr int kDefaultAttnTileBf16 = 14;
int attn_tile_of(const mlpf_model_s* m) {
  if (m->tune[MLPF_OP_ATTENTION] >= 0) return m->tune[MLPF_OP_ATTENTION];
  return m->kprec == P_BF16 ? kDefaultAttnTileBf16 : 0;
}

// Key splits of one attention launch over T rows: the pinned count (MLPF_OP_ATTN_SPLIT), else the
// fewest (a power of two) that give the launch about three waves per SIMD when the rows form one
// event (4 SIMDs x 256 CUs); only the BF16 bound-offset kernels split, within the workspace's cap.
int attn_split_of(const mlpf_model_s* m, const WsPlan& w, int64_t T) {
  const AttnTile at = attn_tile(attn_tile_of(m));
  if (m->kprec != P_BF16 || at.kind < 1 || w.split_cap < 2) return 1;
  int s = 1;
  if (m->tune[MLPF_OP_ATTN_SPLIT] >= 0) {
    s = 1 << m->tune[MLPF_OP_ATTN_SPLIT];
  } else {
    const int64_t qt = 32 * at.waves * at.qb;
    const int64_t waves = (int64_t)m->cfg.n_heads * ((T + qt - 1) / qt) * at.waves;
    while (s < 8 && waves * s < 3 * 4 * 256) s *= 2;
  }
  return std::min(s, w.split_cap);
}

mlpf_status_t run_gemm(const Ctx& cx, int op, ALoad al, Epi ep, GemmArgs a, int prec = -1) {
  a.m_dev = cx.n_rows;
  a.relu = cx.m->cfg.activation == MLPF_ACT_RELU;
  const int pr = prec >= 0 ? prec : (int)cx.m->kprec;
  const int eb = pr == P_F32 ? 4 : pr == P_BF16 ? 2 : 1;
  const int tile = cx.m->tune[op] >= 0 ? cx.m->tune[op] : pick_gemm_tile(a.M, a.N, a.Kp * eb, (Prec)pr);
  HIP_TRY(launch_gemm((Prec)pr, al, ep, tile, a, cx.s), "gemm launch");
  return MLPF_OK;
}

// y = LayerNorm(h) in the operand type (the A operand of the next product).
mlpf_status_t run_layernorm(const Ctx& cx, const void* h, size_t g_off, size_t b_off,
                            int prec = -1, float out_scale = 1.f, float* amax = nullptr) {
  LayerNormArgs a;
  a.out_scale = out_scale;
  a.amax = amax;
  a.x = h;
  a.x_bf16 = cx.m->hbytes == 2;
  a.y = cx.p(cx.w.y);
  a.rows = cx.b->total_rows;
  a.d = cx.m->cfg.d_model;
  a.m_dev = cx.n_rows;
  a.gamma = cx.m->atf(g_off);
  a.beta = cx.m->atf(b_off);
  a.eps = cx.m->cfg.ln_eps;
  HIP_TRY(launch_layernorm(prec >= 0 ? (Prec)prec : cx.m->kprec, a, cx.s), "layernorm launch");
  return MLPF_OK;
}

// One embedding network (W1, b1, W2, b2 at the given plan offsets) over every row, into out.
mlpf_status_t embed_net(const Ctx& cx, const float* x, void* out, size_t w1, size_t b1, size_t w2,
                        size_t b2) {
  const mlpf_model_s* m = cx.m;
  const int T = cx.b->total_rows, d = m->cfg.d_model;
  GemmArgs a;
  a.a = x;
  a.lda = m->cfg.n_features;
  a.M = T;
  a.N = d;
  a.K = m->cfg.n_features;
  a.Kp = kEmbedKp;
  a.wt = m->at(w1);
  a.bias = m->atf(b1);
  a.out = cx.p(cx.w.u);
  a.ldo = d;
  mlpf_status_t st = run_gemm(cx, MLPF_OP_EMBED1, A_SCALAR, E_GELU, a);
  if (st) return st;
  GemmArgs b;
  b.a = cx.p(cx.w.u);
  b.lda = d;
  b.M = T;
  b.N = d;
  b.K = d;
  b.Kp = d;
  b.wt = m->at(w2);
  b.bias = m->atf(b2);
  b.out = out;
  b.ldo = d;
  return run_gemm(cx, MLPF_OP_EMBED2, A_PLAIN, m->hbytes == 2 ? E_BIAS_B : E_BIAS, b);
}

// The embedding (Sec. 5.3). embed_per_type: the track network into h, the other network into the
// LN buffer y (free at this point, rows of the same type and width), then the non-track rows of h
// are replaced from y.
mlpf_status_t do_embed(const Ctx& cx, const float* x, void* h) {
  const mlpf_model_s* m = cx.m;
  ProfScope prof(cx.m, MLPF_PROF_EMBED, cx.s);
  const int T = cx.b->total_rows, d = m->cfg.d_model;
  if (T == 0) return MLPF_OK;
  const WeightPlan& P = m->plan;
  mlpf_status_t st = embed_net(cx, x, h, P.e_w1, P.e_b1, P.e_w2, P.e_b2);
  if (st || !m->cfg.embed_per_type) return st;
  void* y = cx.p(cx.w.y);
  if ((st = embed_net(cx, x, y, P.c_w1, P.c_b1, P.c_w2, P.c_b2))) return st;
  HIP_TRY(launch_select_rows(h, y, x, m->cfg.n_features, T, cx.n_rows, d * m->hbytes, cx.s),
          "embedding select");
  return MLPF_OK;
}

// The sanitised event table, the live row count and the attention work list. With attention
// partitions a second launch lists the work items of the partitions instead (the first one's items
// are overwritten; its row count is the batch's).
mlpf_status_t do_worklist(Ctx& cx) {
  const mlpf_model_s* m = cx.m;
  WorklistArgs a;
  a.row_start = cx.b->row_start;
  a.n_valid = cx.b->n_valid;
  a.n_events = cx.b->n_events;
  a.total_rows = cx.b->total_rows;
  a.max_seqlen = cx.b->max_seqlen;
  const AttnTile at = attn_tile(attn_tile_of(m));
  a.q_tile = 32 * at.waves * at.qb;
  a.n_heads = m->cfg.n_heads;
  a.cap_items = cx.w.cap_items;
  a.ev_start = (int32_t*)cx.p(cx.w.ev_start);
  a.ev_n = (int32_t*)cx.p(cx.w.ev_n);
  a.items = (int32_t*)cx.p(cx.w.items);
  int32_t* ctr = (int32_t*)cx.p(cx.w.counters);
  a.n_items = ctr;
  a.n_rows = ctr + 1;
  {
    ProfScope prof(cx.m, MLPF_PROF_WORKLIST, cx.s);
    HIP_TRY(launch_worklist(a, cx.s), "worklist launch");
    if (const mlpf_batch_t* q = cx.b->attn_parts) {
      a.row_start = q->row_start;
      a.n_valid = q->n_valid;
      a.n_events = q->n_events;
      a.max_seqlen = q->max_seqlen;
      a.n_rows = ctr + 2;  // unused
      HIP_TRY(launch_worklist(a, cx.s), "worklist launch");
    }
  }
  cx.n_rows = ctr + 1;
  return MLPF_OK;
}

// Attention over the work list built by do_worklist; q is pre-scaled by log2(e)/sqrt(d_head).
mlpf_status_t run_attention(const Ctx& cx, const void* q, const void* k, const void* v, void* o,
                            bool knorm_ready = false) {
  const mlpf_model_s* m = cx.m;
  AttnArgs at;
  at.q = q;
  at.k = k;
  at.v = v;
  at.o = o;
  at.hstride = (int64_t)cx.b->total_rows * m->dh;
  at.d = m->cfg.d_model;
  at.dh = m->dh;
  const int32_t* ctr = (const int32_t*)cx.p(cx.w.counters);
  at.items = (const int32_t*)cx.p(cx.w.items);
  at.n_items = ctr;
  at.ev_start = (const int32_t*)cx.p(cx.w.ev_start);
  at.ev_n = (const int32_t*)cx.p(cx.w.ev_n);
  at.cap_items = cx.w.cap_items;
  const int tile = attn_tile_of(m);
  if (m->kprec == P_BF16 && attn_tile(tile).kind >= 1) {
    // Squared key norms for the score bound: written by the QKV projection in the forward pass,
    // computed here for mlpf_attention_forward (timed with the QKV class).
    float* kn = (float*)cx.p(cx.w.knorm);
    if (!knorm_ready) {
      ProfScope prof(cx.m, MLPF_PROF_QKV, cx.s);
      HIP_TRY(launch_keynorm(k, kn, (int64_t)cx.b->total_rows * m->cfg.n_heads, m->dh, cx.s),
              "keynorm launch");
    }
    at.knorm = kn;
  }
  at.rows = cx.b->total_rows;
  at.q_tile = 32 * attn_tile(tile).waves * attn_tile(tile).qb;
  at.ksplit = attn_split_of(m, cx.w, cx.b->total_rows);
  if (at.ksplit > 1) {
    at.part_o = (float*)cx.p(cx.w.part_o);
    at.part_ml = (float*)cx.p(cx.w.part_ml);
  }
  ProfScope prof(cx.m, MLPF_PROF_ATTENTION, cx.s);
  HIP_TRY(launch_attention(m->kprec, tile, at, cx.s), "attention launch");
  if (at.ksplit > 1) HIP_TRY(launch_attn_combine(at, cx.s), "attention combine launch");
  return MLPF_OK;
}

// The fused FFN kernel runs unless the model cannot use it or MLPF_OP_FFN is pinned to 0.
bool ffn_fused_on(const mlpf_model_s* m) {
  return m->plan.ffn_fused && m->tune[MLPF_OP_FFN] != 0;
}

// FFN tiles 5 to 8 and 9 to 12: the 64-row and the 128-row fused shapes with the hidden units in
// 2, 4, 8 or 16 parts.
int ffn_tile_parts(int t) { return t >= 9 ? 1 << (t - 8) : t >= 5 ? 1 << (t - 4) : t > 0; }

// Parts of the hidden units a fused FFN over T rows is split into (the tile's, or the rule's: the
// fewest, a power of two, that give two 64-row workgroups per CU), within the workspace's partial
// buffers and dividing the 64-unit chunk count; 1 = no split.
int ffn_split_of(const mlpf_model_s* m, const WsPlan& w, int64_t T) {
  const int t = m->tune[MLPF_OP_FFN];
  int s = 1;
  if (t >= 5) {
    s = ffn_tile_parts(t);
  } else if (t == -1) {
    const int64_t row_tiles = (T + 63) / 64;
    while (s < 16 && row_tiles * s < 2 * 256) s *= 2;
  }
  s = std::min(s, w.split_cap);
  while (s > 1 && (m->cfg.d_ff / 64) % s) s /= 2;
  return s;
}

// One encoder block. y_ready: y already holds LN1(h) (written by the previous block's fused FFN).
// *y_next_out: set when this block's fused FFN also wrote the next block's LN1 into y.
mlpf_status_t do_layer(const Ctx& cx, int layer, void* h, bool y_ready = false,
                       bool fuse_next_ln = false, bool* y_next_out = nullptr) {
  const mlpf_model_s* m = cx.m;
  const mlpf_config_t& c = m->cfg;
  const Layer& L = m->plan.layers[layer];
  const int T = cx.b->total_rows, d = c.d_model, dh = m->dh;
  mlpf_status_t st;
  // LN1 + QKV projection, head-major Q (scaled by log2(e)/sqrt(d_head)), K, V.
  GemmArgs q;
  q.a = cx.p(cx.w.y);
  q.lda = d;
  q.M = T;
  q.N = 3 * d;
  q.K = d;
  q.Kp = d;
  q.wt = m->at(L.wqkv);
  q.bias = m->atf(L.bqkv);
  q.q = cx.p(cx.w.q);
  q.k = cx.p(cx.w.k);
  q.v = cx.p(cx.w.v);
  q.hstride = (int64_t)T * dh;
  q.d = d;
  q.dh = dh;
  q.q_scale = (float)(1.4426950408889634 / std::sqrt((double)dh));
  // The BF16 score-bound attention reads squared key norms: the projection's epilogue writes them.
  const bool kn_fused = m->kprec == P_BF16 && attn_tile(attn_tile_of(m)).kind >= 1;
  if (kn_fused) q.knorm = (float*)cx.p(cx.w.knorm);
  {
    ProfScope prof(cx.m, MLPF_PROF_QKV, cx.s);
    if (!y_ready && (st = run_layernorm(cx, h, L.ln1g, L.ln1b))) return st;
    if ((st = run_gemm(cx, MLPF_OP_QKV, A_PLAIN, E_QKV, q))) return st;
  }
  // Attention.
  if ((st = run_attention(cx, cx.p(cx.w.q), cx.p(cx.w.k), cx.p(cx.w.v), cx.p(cx.w.o), kn_fused)))
    return st;
  // Output projection + residual.
  GemmArgs o;
  o.a = cx.p(cx.w.o);
  o.lda = d;
  o.M = T;
  o.N = d;
  o.K = d;
  o.Kp = d;
  o.wt = m->at(L.wo);
  o.bias = m->atf(L.bo);
  o.out = h;
  o.ldo = d;
  // LN2 follows the residual update (timed with it); the fused FFN computes it itself from h.
  const bool fp8 = m->prec == MLPF_BF16_FP8FFN;
  const bool ffn_one = ffn_fused_on(m) && !cx.calib;
  float* am1 = cx.calib ? cx.calib + 2 * layer : nullptr;
  float* am2 = cx.calib ? cx.calib + 2 * layer + 1 : nullptr;
  {
    ProfScope prof(cx.m, MLPF_PROF_OUTPROJ, cx.s);
    if ((st = run_gemm(cx, MLPF_OP_OUTPROJ, A_PLAIN, m->hbytes == 2 ? E_RESID_B : E_RESID, o))) return st;
    if (!ffn_one && (st = run_layernorm(cx, h, L.ln2g, L.ln2b, fp8 ? P_FP8 : -1,
                                        fp8 ? 1.f / L.s_a1 : 1.f, am1)))
      return st;
  }
  // LN2 + FFN1 + GELU, FFN2 + residual. FP8 mode: LN2 writes E4M3 (scaled by 1/s_a1), FFN1
  // dequantises with s_a1 s_w1 and writes GELU output as E4M3 (1/s_a2), FFN2 dequantises with
  // s_a2 s_w2.
  GemmArgs f1;
  f1.a = cx.p(cx.w.y);
  f1.lda = d;
  f1.M = T;
  f1.N = c.d_ff;
  f1.K = d;
  f1.Kp = d;
  f1.wt = m->at(L.w1);
  f1.bias = m->atf(L.b1);
  f1.out = cx.p(cx.w.u);
  f1.ldo = c.d_ff;
  f1.amax = am2;
  if (fp8) {
    f1.acc_scale = L.s_a1 * L.s_w1;
    f1.out_scale = 1.f / L.s_a2;
  }
  if (ffn_one) {
    // One kernel: the d_ff-wide intermediate stays on chip (timed in the FFN1 class).
    ProfScope prof(cx.m, MLPF_PROF_FFN1, cx.s);
    FfnArgs a;
    a.y = h;  // LN2 in the kernel
    a.ln_in_g = m->atf(L.ln2g);
    a.ln_in_b = m->atf(L.ln2b);
    a.ln_in_eps = c.ln_eps;
    a.M = T;
    a.m_dev = cx.n_rows;
    a.d_model = d;
    a.d_ff = c.d_ff;
    a.w1p = m->at(L.w1p);
    a.b1 = m->atf(L.b1);
    a.w2p = m->at(L.w2p);
    a.b2 = m->atf(L.b2);
    a.relu = c.activation == MLPF_ACT_RELU;
    a.h = h;
    if (fuse_next_ln) {
      const Layer& Ln = m->plan.layers[layer + 1];
      a.y_next = cx.p(cx.w.y);
      a.ln_g = m->atf(Ln.ln1g);
      a.ln_b = m->atf(Ln.ln1b);
      a.ln_eps = c.ln_eps;
      if (y_next_out) *y_next_out = true;
    }
    if (fp8) {
      a.fp8_in_scale = 1.f / L.s_a1;
      a.acc_scale = L.s_a1 * L.s_w1;
      a.out_scale = 1.f / L.s_a2;
      a.acc_scale2 = L.s_a2 * L.s_w2;
      HIP_TRY(launch_ffn_fp8(a, cx.s), "fused FP8 FFN launch");
      return MLPF_OK;
    }
    const int ffn_default = (c.d_ff / 64) % 2 == 0 ? 4 : 3;  // pipelined when the chunk count is even
    const int tune = m->tune[MLPF_OP_FFN];
    int variant = tune >= 9 ? 1 : tune >= 5 ? 2 : tune > 0 ? tune : ffn_default;
    a.split = ffn_split_of(m, cx.w, T);
    if (a.split > 1) {
      a.part = (float*)cx.p(cx.w.part_o);
      variant = tune >= 9 ? 6 : 5;
    }
    HIP_TRY(launch_ffn_fused(a, variant, cx.s), "fused FFN launch");
    return MLPF_OK;
  }
  {
    ProfScope prof(cx.m, MLPF_PROF_FFN1, cx.s);
    if ((st = run_gemm(cx, MLPF_OP_FFN1, A_PLAIN, E_GELU, f1, fp8 ? P_FP8 : -1))) return st;
  }
  GemmArgs f2;
  f2.a = cx.p(cx.w.u);
  f2.lda = c.d_ff;
  f2.M = T;
  f2.N = d;
  f2.K = c.d_ff;
  f2.Kp = c.d_ff;
  f2.wt = m->at(L.w2);
  f2.bias = m->atf(L.b2);
  f2.out = h;
  f2.ldo = d;
  if (fp8) f2.acc_scale = L.s_a2 * L.s_w2;
  ProfScope prof(cx.m, MLPF_PROF_FFN2, cx.s);
  return run_gemm(cx, MLPF_OP_FFN2, A_PLAIN, m->hbytes == 2 ? E_RESID_B : E_RESID, f2, fp8 ? P_FP8 : -1);
}

mlpf_status_t do_encoder(Ctx& cx, void* h) {
  const mlpf_model_s* m = cx.m;
  const int64_t td = (int64_t)cx.b->total_rows * m->cfg.d_model;
  if (cx.b->total_rows == 0) return MLPF_OK;
  mlpf_status_t st;
  if (!cx.n_rows && (st = do_worklist(cx))) return st;
  if (m->stacks == 1) {
    bool y_ready = false;
    for (int l = 0; l < m->cfg.n_layers; ++l) {
      bool next = false;
      if ((st = do_layer(cx, l, h, y_ready, l + 1 < m->cfg.n_layers, &next))) return st;
      y_ready = next;
    }
  } else {
    void* h1 = (char*)h + td * m->hbytes;
    HIP_TRY(launch_copy_f32((float*)h1, (const float*)h, td * m->hbytes / 4, cx.s), "copy launch");
    const int half = m->cfg.n_layers / 2;
    bool y_ready = false;
    for (int l = 0; l < m->cfg.n_layers; ++l) {
      // The next block's LN1 can only be fused within a stack (stack 1 starts from the embedding).
      const bool same_stack_next = l + 1 < m->cfg.n_layers && l + 1 != half;
      bool next = false;
      if ((st = do_layer(cx, l, l < half ? h : h1, y_ready, same_stack_next, &next))) return st;
      y_ready = next;
    }
  }
  return MLPF_OK;
}

mlpf_status_t do_heads(const Ctx& cx, const void* h, float* logits, float* reg, int32_t* cls,
                       const float* prim, float* decoded) {
  const mlpf_model_s* m = cx.m;
  const int T = cx.b->total_rows, d = m->cfg.d_model;
  if (T == 0) return MLPF_OK;
  const int64_t td = (int64_t)T * d;
  const size_t eb = elem_bytes(m->prec);
  mlpf_status_t st;
  ProfScope prof(cx.m, MLPF_PROF_HEADS, cx.s);
  // First layer of every head: [T][d] -> act -> [T][nh d]. For PARALLEL2 the classification
  // head(s) read stack 0 and the regression heads stack 1.
  const int nh = n_out_heads(m->cfg), ncls = n_cls_heads(m->cfg);
  const int groups = m->stacks == 1 ? 1 : 2;
  // Fused (d_model 256, bf16 operands): 64 x 256 tiles, one head per column tile; the epilogue
  // keeps act(first layer) on chip and writes only the 11 second-layer sums per row (into u).
  const bool fused = m->plan.heads_fused && m->tune[MLPF_OP_HEADS] != 0;
  for (int g = 0; g < groups; ++g) {
    const int c0 = (groups == 1) ? 0 : (g == 0 ? 0 : ncls * d);
    const int nc = (groups == 1) ? nh * d : (g == 0 ? ncls * d : (nh - ncls) * d);
    GemmArgs a;
    a.a = (const char*)h + (g == 0 ? 0 : td * m->hbytes);
    a.lda = d;
    a.M = T;
    a.N = nc;
    a.K = d;
    a.Kp = d;
    a.wt = (const char*)m->at(m->plan.h_w1) + (size_t)c0 * d * eb;
    a.bias = m->atf(m->plan.h_b1) + c0;
    a.out = (char*)cx.p(cx.w.u) + (size_t)c0 * eb;
    a.ldo = nh * d;
    a.heads6 = nh == 6;
    if (fused) {
      a.m_dev = cx.n_rows;
      a.w2 = m->atf(m->plan.h_w2);
      a.hout = (float*)cx.p(cx.w.u);
      a.head0 = c0 / d;
      a.relu = m->cfg.activation == MLPF_ACT_RELU;
      HIP_TRY(launch_gemm(P_BF16, A_PLAIN, E_HEADS, kHeadsTile, a, cx.s), "gemm launch");
      continue;
    }
    if ((st = run_gemm(cx, MLPF_OP_HEADS1, m->hbytes == 2 ? A_PLAIN : A_F32, E_GELU, a))) return st;
  }
  Heads2Args p;
  p.binary = m->cfg.decision == MLPF_DECIDE_BINARY;
  p.heads6 = nh == 6;
  p.uh = cx.p(cx.w.u);
  p.d = d;
  p.rows = T;
  p.m_dev = cx.n_rows;
  p.w2 = m->atf(m->plan.h_w2);
  p.b2 = m->atf(m->plan.h_b2);
  p.logits = logits;
  p.reg = reg;
  p.cls = cls;
  p.prim = prim;
  p.decoded = decoded;
  if (fused) {
    HIP_TRY(launch_heads_finish(p, cx.s), "heads launch");
  } else {
    HIP_TRY(launch_heads2(m->kprec, p, cx.s), "heads launch");
  }
  return MLPF_OK;
}

// Scratch of mlpf_reconstruct_events_noalloc: a fixed-size array in device memory, one copy per
// GPU, held from the library's load until the process ends (each GPU the library runs on holds its
// own). In host code `scratch` names a host-side stand-in, never the device memory: host code uses
// only the device address hipGetSymbolAddress returns, looked up once per device with that device
// current (at mlpf_model_create, or at the entry point's first call on a device).
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

mlpf_status_t scratch_of_current_device(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(MLPF_ERR_UNSUPPORTED, "device %d is beyond the %d devices the scratch table holds",
                dev, kMaxDevices);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address");
    if (!p) return fail(MLPF_ERR_INTERNAL, "no device address for the scratch array");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return MLPF_OK;
}

mlpf_status_t make_ctx(mlpf_model_t m, const mlpf_batch_t* b, void* ws, size_t ws_bytes,
                       void* stream, bool need_h, Ctx* cx) {
  if (!m) return fail(MLPF_ERR_INVALID_ARG, "model is NULL");
  mlpf_status_t st = check_batch(m, b);
  if (st) return st;
  cx->m = m;
  cx->b = b;
  cx->w = plan_ws(m, b->total_rows, std::max(b->n_events, b->attn_parts ? b->attn_parts->n_events : 0));
  const size_t need = need_h ? cx->w.total : cx->w.h;
  if (need > 0 && !ws) return fail(MLPF_ERR_INVALID_ARG, "workspace is NULL");
  if (ws_bytes < need)
    return fail(MLPF_ERR_INVALID_ARG, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  cx->ws = (char*)ws;
  cx->s = (hipStream_t)stream;
  cx->n_rows = nullptr;
  return MLPF_OK;
}

}  // namespace

extern "C" {

size_t mlpf_weights_bytes(const mlpf_config_t* cfg, mlpf_precision_t precision) {
  if (check_config(cfg) != MLPF_OK) return 0;
  if (precision != MLPF_FP32 && precision != MLPF_BF16 && precision != MLPF_BF16_FP8FFN) return 0;
  return plan_weights(*cfg, precision).total;
}

size_t mlpf_weights_count(const mlpf_config_t* cfg) {
  if (check_config(cfg) != MLPF_OK) return 0;
  return master_count(*cfg);
}

mlpf_status_t mlpf_model_create(const mlpf_config_t* cfg, mlpf_precision_t precision,
                                const float* host_weights, size_t n_floats,
                                const float* act_amax, void* dev_weights, size_t dev_bytes,
                                void* stream, mlpf_model_t* out) {
  if (!out) return fail(MLPF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  mlpf_status_t st = check_config(cfg);
  if (st) return st;
  if (precision != MLPF_FP32 && precision != MLPF_BF16 && precision != MLPF_BF16_FP8FFN)
    return fail(MLPF_ERR_INVALID_ARG, "unknown precision %d", (int)precision);
  if (precision == MLPF_BF16_FP8FFN) {
    if (!act_amax) return fail(MLPF_ERR_INVALID_ARG, "MLPF_BF16_FP8FFN needs act_amax");
    for (int i = 0; i < 2 * cfg->n_layers; ++i)
      if (!(act_amax[i] >= 0.f) || !std::isfinite(act_amax[i]))
        return fail(MLPF_ERR_INVALID_ARG, "act_amax[%d] must be non-negative and finite", i);
  }
  if (!host_weights) return fail(MLPF_ERR_INVALID_ARG, "host_weights is NULL");
  if (n_floats != master_count(*cfg))
    return fail(MLPF_ERR_INVALID_ARG, "n_floats=%zu, expected %zu", n_floats, master_count(*cfg));
  WeightPlan plan = plan_weights(*cfg, precision);
  if (!dev_weights) return fail(MLPF_ERR_INVALID_ARG, "dev_weights is NULL");
  if (dev_bytes < plan.total)
    return fail(MLPF_ERR_INVALID_ARG, "dev_bytes=%zu < %zu", dev_bytes, plan.total);

  // Pack on the host: Linear weights transposed to [out][in] in the operand type.
  const mlpf_config_t& c = *cfg;
  const int d = c.d_model, f = c.n_features, ff = c.d_ff;
  std::vector<unsigned char> img(plan.total, 0);
  const float* src = host_weights;
  auto put_f32 = [&](size_t off, int n) {
    memcpy(img.data() + off, src, (size_t)n * 4);
    src += n;
  };
  // W is [in][out] in the blob; writes W^T [out][kp] (kp >= in, zero padded).
  auto put_wt = [&](size_t off, int in, int outn, int kp) {
    for (int i = 0; i < in; ++i)
      for (int o = 0; o < outn; ++o) {
        const float v = src[(size_t)i * outn + o];
        const size_t idx = (size_t)o * kp + i;
        if (precision == MLPF_FP32)
          memcpy(img.data() + off + idx * 4, &v, 4);
        else {
          const uint16_t b = f32_to_bf16_rne(v);
          memcpy(img.data() + off + idx * 2, &b, 2);
        }
      }
    src += (size_t)in * outn;
  };
  // FP8 E4M3 with a per-tensor scale amax / 448; returns the scale.
  auto put_wt_fp8 = [&](size_t off, int in, int outn, int kp) {
    float amax = 0.f;
    for (size_t i = 0; i < (size_t)in * outn; ++i) amax = std::max(amax, std::fabs(src[i]));
    const float scale = fp8_scale(amax);
    for (int i = 0; i < in; ++i)
      for (int o = 0; o < outn; ++o)
        img[off + (size_t)o * kp + i] = f32_to_e4m3(src[(size_t)i * outn + o] / scale);
    src += (size_t)in * outn;
    return scale;
  };
  put_wt(plan.e_w1, f, d, kEmbedKp);
  put_f32(plan.e_b1, d);
  put_wt(plan.e_w2, d, d, d);
  put_f32(plan.e_b2, d);
  if (c.embed_per_type) {
    put_wt(plan.c_w1, f, d, kEmbedKp);
    put_f32(plan.c_b1, d);
    put_wt(plan.c_w2, d, d, d);
    put_f32(plan.c_b2, d);
  }
  for (int l = 0; l < c.n_layers; ++l) {
    const Layer L = plan.layers[l];
    put_f32(L.ln1g, d);
    put_f32(L.ln1b, d);
    put_wt(L.wqkv, d, 3 * d, d);
    put_f32(L.bqkv, 3 * d);
    put_wt(L.wo, d, d, d);
    put_f32(L.bo, d);
    put_f32(L.ln2g, d);
    put_f32(L.ln2b, d);
    if (precision == MLPF_BF16_FP8FFN) {
      Layer& Lm = plan.layers[l];
      Lm.s_w1 = put_wt_fp8(L.w1, d, ff, d);
      put_f32(L.b1, ff);
      Lm.s_w2 = put_wt_fp8(L.w2, ff, d, ff);
      put_f32(L.b2, d);
      Lm.s_a1 = fp8_scale(act_amax[2 * l]);
      Lm.s_a2 = fp8_scale(act_amax[2 * l + 1]);
      if (plan.ffn_fused)
        ffn_fp8_pack(img.data() + L.w1, img.data() + L.w2, d, ff, img.data() + L.w1p, img.data() + L.w2p);
    } else {
      put_wt(L.w1, d, ff, d);
      put_f32(L.b1, ff);
      put_wt(L.w2, ff, d, ff);
      put_f32(L.b2, d);
      if (plan.ffn_fused)
        ffn_pack((const uint16_t*)(img.data() + L.w1), (const uint16_t*)(img.data() + L.w2), d, ff,
                 (uint16_t*)(img.data() + L.w1p), (uint16_t*)(img.data() + L.w2p));
    }
  }
  // Heads: W1 of the heads stacked as rows of W^T [nh d][d]; W2 as [d][11] (block diagonal: each
  // output column reads its own head's hidden units).
  const int* widths = head_widths(c);
  const size_t eb = elem_bytes(precision);
  std::vector<float> w2(d * 11, 0.f), b2(11, 0.f);
  int col = 0;
  for (int k = 0; k < n_out_heads(c); ++k) {
    put_wt(plan.h_w1 + (size_t)k * d * d * eb, d, d, d);
    put_f32(plan.h_b1 + (size_t)k * d * 4, d);
    for (int j = 0; j < d; ++j)
      for (int o = 0; o < widths[k]; ++o) w2[(size_t)j * 11 + col + o] = src[(size_t)j * widths[k] + o];
    src += (size_t)d * widths[k];
    for (int o = 0; o < widths[k]; ++o) b2[col + o] = src[o];
    src += widths[k];
    col += widths[k];
  }
  memcpy(img.data() + plan.h_w2, w2.data(), w2.size() * 4);
  memcpy(img.data() + plan.h_b2, b2.data(), b2.size() * 4);
  if ((size_t)(src - host_weights) != n_floats)
    return fail(MLPF_ERR_INTERNAL, "weight packing consumed %zu of %zu floats",
                (size_t)(src - host_weights), n_floats);

  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(dev_weights, img.data(), plan.total, hipMemcpyHostToDevice, s),
          "weight upload");
  HIP_TRY(hipStreamSynchronize(s), "weight upload sync");
  // Set-up of the allocation-free entry point's scratch address on this device (a failure here is
  // reported by that entry point, which looks the address up again).
  void* scratch_dev = nullptr;
  (void)scratch_of_current_device(&scratch_dev);

  mlpf_model_s* m = new (std::nothrow) mlpf_model_s();
  if (!m) return fail(MLPF_ERR_INTERNAL, "out of host memory");
  m->cfg = c;
  m->prec = precision;
  m->kprec = precision == MLPF_FP32 ? P_F32 : P_BF16;
  m->dh = d / c.n_heads;
  m->stacks = c.topology == MLPF_TOPO_PARALLEL2 ? 2 : 1;
  m->hbytes = precision == MLPF_FP32 ? 4 : 2;
  m->plan = plan;
  m->base = (const char*)dev_weights;
  for (int& t : m->tune) t = -1;
  *out = m;
  return MLPF_OK;
}

mlpf_status_t mlpf_model_destroy(mlpf_model_t model) {
  if (model)
    for (auto& v : model->prof_events)
      for (auto& pr : v) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
      }
  delete model;
  return MLPF_OK;
}

size_t mlpf_workspace_bytes(mlpf_model_t model, int32_t total_rows, int32_t max_seqlen,
                            int32_t n_events) {
  if (!model || total_rows < 0 || n_events < 0 || max_seqlen < 0 || max_seqlen > MLPF_MAX_SEQLEN)
    return 0;
  return plan_ws(model, total_rows, n_events).total;
}

mlpf_status_t mlpf_embed(mlpf_model_t model, const float* x, const mlpf_batch_t* batch, void* h,
                         void* ws, size_t ws_bytes, void* stream) {
  Ctx cx;
  mlpf_status_t st = make_ctx(model, batch, ws, ws_bytes, stream, false, &cx);
  if (st) return st;
  if (batch->total_rows > 0 && (!x || !h)) return fail(MLPF_ERR_INVALID_ARG, "x or h is NULL");
  return do_embed(cx, x, h);
}

mlpf_status_t mlpf_encoder_forward(mlpf_model_t model, void* h, const mlpf_batch_t* batch,
                                   void* ws, size_t ws_bytes, void* stream) {
  Ctx cx;
  mlpf_status_t st = make_ctx(model, batch, ws, ws_bytes, stream, false, &cx);
  if (st) return st;
  if (batch->total_rows > 0 && !h) return fail(MLPF_ERR_INVALID_ARG, "h is NULL");
  return do_encoder(cx, h);
}

mlpf_status_t mlpf_heads(mlpf_model_t model, const void* h, const mlpf_batch_t* batch,
                         float* logits, float* reg, int32_t* cls, const float* prim,
                         float* decoded, void* ws, size_t ws_bytes, void* stream) {
  Ctx cx;
  mlpf_status_t st = make_ctx(model, batch, ws, ws_bytes, stream, false, &cx);
  if (st) return st;
  if (batch->total_rows > 0 && (!h || !logits || !reg || !cls))
    return fail(MLPF_ERR_INVALID_ARG, "h, logits, reg or cls is NULL");
  return do_heads(cx, h, logits, reg, cls, prim, decoded);
}

mlpf_status_t mlpf_reconstruct_events(mlpf_model_t model, const float* x,
                                      const mlpf_batch_t* batch, float* logits, float* reg,
                                      int32_t* cls, const float* prim, float* decoded, void* ws,
                                      size_t ws_bytes, void* stream) {
  Ctx cx;
  mlpf_status_t st = make_ctx(model, batch, ws, ws_bytes, stream, true, &cx);
  if (st) return st;
  if (batch->total_rows == 0) return MLPF_OK;
  if (!x || !logits || !reg || !cls) return fail(MLPF_ERR_INVALID_ARG, "x or an output is NULL");
  void* h = cx.p(cx.w.h);
  // The work list first: it also yields the live row count that lets every kernel skip rows
  // beyond the last event (a captured graph sized for a capacity then does no dead work).
  if ((st = do_worklist(cx))) return st;
  if ((st = do_embed(cx, x, h))) return st;
  if ((st = do_encoder(cx, h))) return st;
  return do_heads(cx, h, logits, reg, cls, prim, decoded);
}

mlpf_status_t mlpf_candidates(const mlpf_batch_t* batch, const int32_t* cls, const float* decoded,
                              int32_t* event_offsets, int32_t* cand_row, int32_t* cand_cls,
                              float* cand_kin, int32_t cap, void* stream) {
  mlpf_status_t st = check_batch(nullptr, batch);
  if (st) return st;
  if (!event_offsets) return fail(MLPF_ERR_INVALID_ARG, "event_offsets is NULL");
  if (batch->total_rows > 0 && !cls) return fail(MLPF_ERR_INVALID_ARG, "cls is NULL");
  if (cap < 0) return fail(MLPF_ERR_INVALID_ARG, "negative cap");
  if (cap > 0 && (!cand_row || !cand_cls))
    return fail(MLPF_ERR_INVALID_ARG, "cand_row or cand_cls is NULL");
  if (cand_kin && !decoded) return fail(MLPF_ERR_INVALID_ARG, "cand_kin needs decoded");
  if ((cand_kin && ((uintptr_t)cand_kin % 16 != 0)) || (decoded && ((uintptr_t)decoded % 16 != 0)))
    return fail(MLPF_ERR_INVALID_ARG, "cand_kin and decoded must be 16-byte aligned");
  CandArgs a;
  a.row_start = batch->row_start;
  a.n_valid = batch->n_valid;
  a.n_events = batch->n_events;
  a.total_rows = batch->total_rows;
  a.max_seqlen = batch->max_seqlen;
  a.cls = cls;
  a.decoded = decoded;
  a.offsets = event_offsets;
  a.cand_row = cand_row;
  a.cand_cls = cand_cls;
  a.cand_kin = cand_kin;
  a.cap = cap;
  HIP_TRY(launch_candidates(a, (hipStream_t)stream), "candidate launch");
  return MLPF_OK;
}

mlpf_status_t mlpf_reconstruct_events_noalloc(mlpf_model_t model, const float* x,
                                              const mlpf_batch_t* batch, float* logits, float* reg,
                                              int32_t* cls, const float* prim, float* decoded,
                                              void* stream) {
  if (!model) return fail(MLPF_ERR_INVALID_ARG, "model is NULL");
  mlpf_status_t st = check_batch(model, batch);
  if (st) return st;
  const size_t need =
      plan_ws(model, batch->total_rows,
              std::max(batch->n_events, batch->attn_parts ? batch->attn_parts->n_events : 0)).total;
  if (need > kNoAllocScratchBytes)
    return fail(MLPF_ERR_CAPACITY, "the batch needs %zu bytes of scratch, above the %zu bytes of the "
                "allocation-free entry point", need, kNoAllocScratchBytes);
  void* ws = nullptr;
  if ((st = scratch_of_current_device(&ws))) return st;
  return mlpf_reconstruct_events(model, x, batch, logits, reg, cls, prim, decoded, ws,
                                 kNoAllocScratchBytes, stream);
}

struct mlpf_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

mlpf_status_t mlpf_graph_create(mlpf_model_t model, const float* x, const mlpf_batch_t* batch,
                                float* logits, float* reg, int32_t* cls, const float* prim,
                                float* decoded, void* ws, size_t ws_bytes, void* stream,
                                mlpf_graph_t* out) {
  if (!out) return fail(MLPF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!stream) return fail(MLPF_ERR_INVALID_ARG, "graph capture needs a non-default stream");
  if (!model) return fail(MLPF_ERR_INVALID_ARG, "model is NULL");
  if (model->prof_on) return fail(MLPF_ERR_INVALID_ARG, "disable the profiler before capturing");
  Ctx cx;
  mlpf_status_t st = make_ctx(model, batch, ws, ws_bytes, stream, true, &cx);
  if (st) return st;
  if (batch->total_rows == 0) return fail(MLPF_ERR_INVALID_ARG, "empty capacity");
  if (!x || !logits || !reg || !cls) return fail(MLPF_ERR_INVALID_ARG, "x or an output is NULL");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
  st = mlpf_reconstruct_events(model, x, batch, logits, reg, cls, prim, decoded, ws, ws_bytes,
                               stream);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(s, &g);
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (ec != hipSuccess) return hip_fail(ec, "end capture");
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(ei, "graph instantiate");
  }
  mlpf_graph_s* gr = new (std::nothrow) mlpf_graph_s();
  if (!gr) {
    (void)hipGraphExecDestroy(ex);
    (void)hipGraphDestroy(g);
    return fail(MLPF_ERR_INTERNAL, "out of host memory");
  }
  gr->graph = g;
  gr->exec = ex;
  *out = gr;
  return MLPF_OK;
}

mlpf_status_t mlpf_graph_launch(mlpf_graph_t graph, void* stream) {
  if (!graph) return fail(MLPF_ERR_INVALID_ARG, "graph is NULL");
  HIP_TRY(hipGraphLaunch(graph->exec, (hipStream_t)stream), "graph launch");
  return MLPF_OK;
}

mlpf_status_t mlpf_graph_destroy(mlpf_graph_t graph) {
  if (!graph) return MLPF_OK;
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  delete graph;
  return MLPF_OK;
}

int32_t mlpf_tune_count(int32_t op) {
  if (op < 0 || op >= MLPF_OP_COUNT) return 0;
  if (op == MLPF_OP_FFN) return 13;
  if (op == MLPF_OP_HEADS) return 2;
  if (op == MLPF_OP_ATTN_SPLIT) return 4;
  return op == MLPF_OP_ATTENTION ? attn_num_tiles() : gemm_num_tiles();
}

mlpf_status_t mlpf_tune_set(mlpf_model_t model, int32_t op, int32_t tile) {
  if (!model) return fail(MLPF_ERR_INVALID_ARG, "model is NULL");
  if (op < 0 || op >= MLPF_OP_COUNT) return fail(MLPF_ERR_INVALID_ARG, "op=%d out of range", op);
  if (tile < -1 || tile >= mlpf_tune_count(op))
    return fail(MLPF_ERR_INVALID_ARG, "tile=%d out of range for op %d", tile, op);
  if (op == MLPF_OP_FFN && tile >= 1 && !model->plan.ffn_fused)
    return fail(MLPF_ERR_UNSUPPORTED, "the fused FFN needs a BF16 or FP8 model with d_model 64, 128 or 256");
  if (op == MLPF_OP_FFN && tile >= 5 && (model->cfg.d_ff / 64) % ffn_tile_parts(tile) != 0)
    return fail(MLPF_ERR_UNSUPPORTED, "the split FFN needs d_ff / 64 divisible by its part count %d",
                ffn_tile_parts(tile));
  if (op == MLPF_OP_FFN && tile == 4 && (model->cfg.d_ff / 64) % 2 != 0)
    return fail(MLPF_ERR_UNSUPPORTED, "the pipelined fused FFN needs d_ff a multiple of 128");
  if (op == MLPF_OP_HEADS && tile == 1 && !model->plan.heads_fused)
    return fail(MLPF_ERR_UNSUPPORTED, "the fused heads need a bf16 model with d_model 256");
  model->tune[op] = tile;
  return MLPF_OK;
}

int32_t mlpf_tune_get(mlpf_model_t model, int32_t op) {
  if (!model || op < 0 || op >= MLPF_OP_COUNT) return -1;
  return model->tune[op];
}

mlpf_status_t mlpf_tune_shape(int32_t op, int32_t tile, int32_t* shape) {
  if (!shape) return fail(MLPF_ERR_INVALID_ARG, "shape is NULL");
  if (op < 0 || op >= MLPF_OP_COUNT) return fail(MLPF_ERR_INVALID_ARG, "op=%d out of range", op);
  if (tile < 0 || tile >= mlpf_tune_count(op))
    return fail(MLPF_ERR_INVALID_ARG, "tile=%d out of range for op %d", tile, op);
  if (op == MLPF_OP_ATTENTION) {
    const AttnTile t = attn_tile(tile);
    const int32_t v[6] = {t.waves, t.kt, t.qb, t.kind, 0, 0};
    for (int i = 0; i < 6; ++i) shape[i] = v[i];
  } else if (op == MLPF_OP_ATTN_SPLIT) {
    const int32_t v[6] = {1 << tile, 0, 0, 0, 0, 0};
    for (int i = 0; i < 6; ++i) shape[i] = v[i];
  } else if (op == MLPF_OP_HEADS) {
    const GemmTile t = gemm_tile(kHeadsTile);
    const int32_t v[6] = {tile, tile ? t.bm : 0, tile ? t.bn : 0, 0, 0, 0};
    for (int i = 0; i < 6; ++i) shape[i] = v[i];
  } else if (op == MLPF_OP_FFN) {
    const bool narrow = tile == 2 || (tile >= 5 && tile <= 8);  // 64 rows, 4 waves, single-buffered
    const int rows = narrow ? 64 : tile > 0 ? 128 : 0, waves = narrow ? 4 : tile > 0 ? 8 : 0;
    const int parts = ffn_tile_parts(tile);
    const int32_t v[6] = {parts, rows, waves, tile != 0 && !narrow, tile == 3 || tile == 4, tile == 4};
    for (int i = 0; i < 6; ++i) shape[i] = v[i];
  } else {
    const GemmTile t = gemm_tile(tile);
    const int32_t v[6] = {t.bm, t.bn, t.wm, t.wn, t.bkb, t.persist};
    for (int i = 0; i < 6; ++i) shape[i] = v[i];
  }
  return MLPF_OK;
}

mlpf_status_t mlpf_profiler_enable(mlpf_model_t model, int enable) {
  if (!model) return fail(MLPF_ERR_INVALID_ARG, "model is NULL");
  std::lock_guard<std::mutex> g(model->prof_mu);
  model->prof_on = enable != 0;
  for (auto& u : model->prof_used) u = 0;
  return MLPF_OK;
}

mlpf_status_t mlpf_profiler_read(mlpf_model_t model, int kernel_class, double* total_ms,
                                 int64_t* launches) {
  if (!model || !total_ms || !launches) return fail(MLPF_ERR_INVALID_ARG, "NULL argument");
  if (kernel_class < 0 || kernel_class >= MLPF_PROF_CLASSES)
    return fail(MLPF_ERR_INVALID_ARG, "kernel_class=%d out of range", kernel_class);
  std::lock_guard<std::mutex> g(model->prof_mu);
  double tot = 0.0;
  const size_t used = model->prof_used[kernel_class];
  for (size_t i = 0; i < used; ++i) {
    float ms = 0.f;
    const auto& pr = model->prof_events[kernel_class][i];
    HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second), "profiler event");
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)used;
  return MLPF_OK;
}

mlpf_status_t mlpf_calibrate_fp8(mlpf_model_t model, const float* x, const mlpf_batch_t* batch,
                                 float* amax, void* ws, size_t ws_bytes, void* stream) {
  Ctx cx;
  mlpf_status_t st = make_ctx(model, batch, ws, ws_bytes, stream, true, &cx);
  if (st) return st;
  if (model->prec == MLPF_BF16_FP8FFN)
    return fail(MLPF_ERR_INVALID_ARG, "calibrate with an FP32 or BF16 model");
  if (batch->total_rows == 0) return MLPF_OK;
  if (!x || !amax) return fail(MLPF_ERR_INVALID_ARG, "x or amax is NULL");
  cx.calib = amax;
  void* h = cx.p(cx.w.h);
  if ((st = do_worklist(cx))) return st;
  if ((st = do_embed(cx, x, h))) return st;
  return do_encoder(cx, h);
}

mlpf_status_t mlpf_attention_forward(mlpf_model_t model, const void* q, const void* k,
                                     const void* v, void* o, const mlpf_batch_t* batch, void* ws,
                                     size_t ws_bytes, void* stream) {
  Ctx cx;
  mlpf_status_t st = make_ctx(model, batch, ws, ws_bytes, stream, false, &cx);
  if (st) return st;
  if (batch->total_rows == 0) return MLPF_OK;
  if (!q || !k || !v || !o) return fail(MLPF_ERR_INVALID_ARG, "q, k, v or o is NULL");
  if ((st = do_worklist(cx))) return st;
  const int64_t n = (int64_t)batch->total_rows * model->cfg.d_model;
  const float scale = (float)(1.4426950408889634 / std::sqrt((double)model->dh));
  HIP_TRY(launch_scale(model->kprec, cx.p(cx.w.q), q, n, scale, cx.s), "scale launch");
  return run_attention(cx, cx.p(cx.w.q), k, v, o);
}

const char* mlpf_status_string(mlpf_status_t s) {
  switch (s) {
    case MLPF_OK: return "MLPF_OK";
    case MLPF_ERR_INVALID_ARG: return "MLPF_ERR_INVALID_ARG";
    case MLPF_ERR_UNSUPPORTED: return "MLPF_ERR_UNSUPPORTED";
    case MLPF_ERR_CAPACITY: return "MLPF_ERR_CAPACITY";
    case MLPF_ERR_HIP: return "MLPF_ERR_HIP";
    case MLPF_ERR_INTERNAL: return "MLPF_ERR_INTERNAL";
  }
  return "unknown status";
}

const char* mlpf_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
