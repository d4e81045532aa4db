/*
 * mlpf.h - C ABI of libmlpf, an MI355X (gfx950) implementation of the MLPF forward pass:
 * the transformer that maps each collision event's set of PF elements (tracks and calorimeter
 * clusters) to per-element particle outputs (arxiv 2601.17554, Sec. 5.3).
 *
 * Model (Sec. 5.3, with the readings stated below):
 *   h0      = act(x W_e1 + b_e1) W_e2 + b_e2                          element embedding FFN
 *   block   : h += MHA(LN1(h));  h += act(LN2(h) W_1 + b_1) W_2 + b_2    pre-LN transformer block
 *   MHA     : per head, softmax(Q K^T / sqrt(d_head)) V over the event's own elements (Eq. 4)
 *   heads   : out_k = act(h W_k1 + b_k1) W_k2 + b_k2, two-layer heads: either five heads
 *             cls(6), pT'(1), eta(1), phi(2), E'(1), or the paper's six (binary_head): binary(1),
 *             particle type(5), pT'(1), eta(1), phi(2), E'(1)
 *   class   = from the six classification outputs by the config's decision rule (mlpf_decision_t)
 *   decode  : pT = pT_prim exp(pT'), E = E_prim exp(E') (inverse of Eq. 2), phi = atan2(sin, cos)
 * act is GELU (default) or ReLU (the paper's network) after every hidden linear layer, none after
 * output layers. GELU(z) = z (1 + erf(z / sqrt 2)) / 2: in MLPF_FP32 with erf evaluated by the
 * Abramowitz-Stegun rational approximation 7.1.26 (absolute error of erf at most 1.5e-7); in the
 * BF16 and FP8 modes, whose hidden activations are rounded to bf16 or E4M3, as z sigma(g(z)) with
 * g an odd quintic fitted to the normal CDF (absolute error of the CDF at most 1.9e-5, of GELU
 * 5.5e-5).
 * Readings where the paper is silent: LayerNorm eps from the config, biased variance; no final
 * LayerNorm; Q/K/V/O biases; contiguous head split.
 *
 * Conventions for every call:
 *   - All pointers to tensors are DEVICE pointers unless a parameter says "host". The caller owns
 *     all memory; the library never allocates device memory and never frees it. Only
 *     mlpf_model_create synchronises its stream (after the weight upload); no other call does.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream). Work is enqueued on it
 *     in order; errors of kernels that already ran surface at the caller's next synchronisation.
 *   - Arguments are validated before anything is enqueued. On failure nothing is written and the
 *     call returns a status; mlpf_last_error() gives a message (thread-local).
 *   - Row-major layouts. Rows of all events are packed one after another ("varlen"); see
 *     mlpf_batch_t. Padding rows (rows of an event beyond its valid count) are never attention
 *     keys; their outputs are unspecified and must be ignored.
 *   - Calls on distinct streams with distinct workspaces and outputs may run concurrently on one
 *     model handle; the handle is immutable after creation.
 */
#ifndef MLPF_H
#define MLPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLPF_N_CLASSES 6     /* classification logits per element */
#define MLPF_N_REG 5         /* pT', eta, sin phi, cos phi, E' per element */
#define MLPF_MAX_SEQLEN 8192 /* largest supported element count of one event */

typedef enum {
  MLPF_OK = 0,
  MLPF_ERR_INVALID_ARG = 1, /* null pointer, inconsistent sizes, workspace too small, ... */
  MLPF_ERR_UNSUPPORTED = 2, /* valid but not supported (e.g. max_seqlen > 8192, d_head not 16/32) */
  MLPF_ERR_CAPACITY = 3,    /* a size exceeds a capacity fixed at creation */
  MLPF_ERR_HIP = 4,         /* a HIP runtime call failed; the message holds the HIP error string */
  MLPF_ERR_INTERNAL = 5
} mlpf_status_t;

/* Arithmetic of the matrix products. Softmax statistics, LayerNorm statistics, every accumulation
 * and all outputs are FP32 in every mode; the residual stream h is FP32 in MLPF_FP32 and bf16 in
 * the BF16 modes (see mlpf_embed); nothing uses FP64 on the GPU. */
typedef enum {
  MLPF_FP32 = 0,        /* FP32 operands on FP32 MFMA */
  MLPF_BF16 = 1,        /* BF16 operands, FP32 accumulation */
  MLPF_BF16_FP8FFN = 2  /* as BF16, but both FFN products take FP8-E4M3 operands with
                           per-tensor scales amax/448 (weights: their own amax; activations: the
                           calibrated act_amax of mlpf_model_create) */
} mlpf_precision_t;

typedef enum {
  MLPF_TOPO_SERIAL = 0,   /* one stack of n_layers blocks; every head reads its output */
  MLPF_TOPO_PARALLEL2 = 1 /* the paper's form (Sec. 5.3): two stacks fed by the same embedding;
                             blocks 0..L/2-1 feed the classification head, blocks L/2..L-1 the
                             regression heads */
} mlpf_topology_t;

/* The hidden-layer activation: the erf GELU (evaluated as stated above), or ReLU as in the paper's
 * network (Sec. 5.3). */
typedef enum { MLPF_ACT_GELU = 0, MLPF_ACT_RELU = 1 } mlpf_activation_t;
/* The class rule (Sec. 5.3). ARGMAX: cls = argmax of the six logits, class 0 = no particle.
 * BINARY: output 0 is a binary "is a particle" logit and outputs 1..5 the particle-type logits;
 * cls = 0 unless sigmoid(output 0) > 0.5 (output 0 > 0), else 1 + argmax of outputs 1..5. Ties go
 * to the lowest index in both. */
typedef enum { MLPF_DECIDE_ARGMAX = 0, MLPF_DECIDE_BINARY = 1 } mlpf_decision_t;

typedef struct {
  int32_t n_features; /* F: features per element, 1..32 */
  int32_t d_model;    /* d: multiple of 64, 64..1024 */
  int32_t n_heads;    /* d / n_heads must be 16 or 32 */
  int32_t d_ff;       /* FFN width: multiple of 64, 64..4096 */
  int32_t n_layers;   /* >= 1; even for MLPF_TOPO_PARALLEL2 */
  int32_t topology;   /* mlpf_topology_t */
  float ln_eps;       /* LayerNorm epsilon (> 0) */
  int32_t activation; /* mlpf_activation_t: after every hidden linear layer (embedding, FFN, heads) */
  int32_t decision;   /* mlpf_decision_t: how cls is taken from the six classification outputs */
  int32_t embed_per_type; /* 0: one embedding network; 1: tracks (feature 0 > 0.5, the one-hot of
                           * element type 0) use the embedding network, every other element a
                           * second one of the same shape (the paper's separate track and cluster
                           * embeddings, Sec. 5.3) */
  int32_t binary_head; /* 0: one classification head with six outputs; 1: the paper's two
                        * classification heads (Sec. 5.3 and its model figure): a binary head
                        * (one output) and a particle-type head (five outputs), each a two-layer
                        * FFN on the classification encoder; the six logits are then
                        * (binary, type 1..5) */
} mlpf_config_t;

typedef struct mlpf_model_s* mlpf_model_t;

/* One launch processes n_events events packed row-wise. Event e owns rows
 * row_start[e] .. row_start[e+1]-1; the first n_valid[e] of them are its elements, the rest are
 * padding. Device arrays are read by the kernels; host sizes bound the launch.
 * Host mirrors (optional): when row_start_host is non-NULL it must hold the same values as the
 * device row_start (and n_valid_host those of n_valid, required then whenever n_valid is
 * non-NULL); the call validates them before anything is enqueued and returns
 * MLPF_ERR_INVALID_ARG with nothing written for row_start_host[0] < 0, a decreasing row_start,
 * row_start_host[n_events] > total_rows, an n_valid outside 0 .. its event's row span, or a valid
 * count above max_seqlen. Without mirrors the device values are not checked on the host: the
 * kernels clamp out-of-range values into [0, total_rows] and to max_seqlen, so bad offsets cannot
 * make a kernel touch memory outside the caller's buffers (they give wrong, not unsafe, results). */
typedef struct mlpf_batch_s {
  const int32_t* row_start;      /* device, [n_events + 1], non-decreasing, last <= total_rows */
  const int32_t* n_valid;        /* device, [n_events], or NULL: every row of an event is valid */
  const int32_t* row_start_host; /* host mirror of row_start, or NULL */
  const int32_t* n_valid_host;   /* host mirror of n_valid, or NULL */
  int32_t n_events;              /* >= 0 */
  int32_t total_rows;            /* T: rows of x, h and the outputs (>= row_start[n_events]) */
  int32_t max_seqlen;            /* upper bound of every event's valid count; 0..8192 */
  /* Partitioned attention (the paper's closing remark in Sec. 5.3 on partitioning the event before
   * the correlation-building layers; block attention, Sec. 9), or NULL. When set, it describes
   * the attention partitions in the same form over the same rows (total_rows equal, its own
   * attn_parts NULL): partition p is rows row_start[p] .. row_start[p] + n_valid[p] - 1, and every
   * attention layer gives an element as keys only the elements of its partition (everything else
   * acts on each element alone and is unchanged). The partitions must tile each event's valid rows,
   * in order and inside the event (valid rows in no partition get unspecified outputs); with host
   * mirrors on the batch the partitions need theirs too, and the tiling is validated
   * (MLPF_ERR_INVALID_ARG, nothing enqueued). Workspace sizes then take n_events as the larger of
   * the events and the partitions. */
  const struct mlpf_batch_s* attn_parts;
} mlpf_batch_t;

/* Bytes of the device weight buffer for (cfg, precision). */
size_t mlpf_weights_bytes(const mlpf_config_t* cfg, mlpf_precision_t precision);

/* Number of FP32 values of the host master weight blob for cfg. The blob is the concatenation,
 * in this order, of row-major arrays with Linear weights stored [in][out] (y = x W + b):
 *   embed: W1[F][d], b1[d], W2[d][d], b2[d]
 *   only with embed_per_type: the second (non-track) embedding, W1[F][d], b1[d], W2[d][d], b2[d]
 *   for each layer: ln1_gamma[d], ln1_beta[d], W_qkv[d][3d], b_qkv[3d], W_o[d][d], b_o[d],
 *                   ln2_gamma[d], ln2_beta[d], W_1[d][d_ff], b_1[d_ff], W_2[d_ff][d], b_2[d]
 *   heads cls, pt, eta, phi, e (widths 6, 1, 1, 2, 1), or with binary_head the six heads
 *   binary, pid, pt, eta, phi, e (widths 1, 5, 1, 1, 2, 1): W1[d][d], b1[d], W2[d][w], b2[w]
 * W_qkv columns are [Q | K | V], each split into contiguous head slices of d/n_heads. */
size_t mlpf_weights_count(const mlpf_config_t* cfg);

/* Creates a model handle. Packs `host_weights` (host, n_floats FP32 values, order above) into the
 * caller's device buffer `dev_weights` (dev_bytes >= mlpf_weights_bytes) with a copy enqueued on
 * `stream`, and synchronises `stream` once the copy is done; host_weights may be freed when the
 * call returns. act_amax (host, or NULL) is needed only for MLPF_BF16_FP8FFN: 2 floats per layer,
 * the calibrated max |value| of the FFN1 input (the LN2 output) and of the FFN2 input (the
 * activation output) of each block (as accumulated by mlpf_calibrate_fp8); the library takes each
 * per-tensor scale as amax / 448 (1 for an amax of 0). The handle borrows dev_weights (which must
 * outlive it) and holds a small host struct. */
mlpf_status_t mlpf_model_create(const mlpf_config_t* cfg, mlpf_precision_t precision,
                                const float* host_weights, size_t n_floats,
                                const float* act_amax, void* dev_weights, size_t dev_bytes,
                                void* stream, mlpf_model_t* out);
mlpf_status_t mlpf_model_destroy(mlpf_model_t model); /* does not touch dev_weights */

/* Bytes of the workspace needed by any call below for a batch of at most total_rows rows, at most
 * n_events events (or attention partitions, whichever is larger) and valid counts of at most
 * max_seqlen (0 for a NULL model, negative sizes or max_seqlen above 8192). A workspace may be
 * reused by consecutive calls on one stream. */
size_t mlpf_workspace_bytes(mlpf_model_t model, int32_t total_rows, int32_t max_seqlen,
                            int32_t n_events);

/* The residual stream h ([S][T][d] below) is held in the model's activation type: FP32 for
 * MLPF_FP32, bf16 (raw 16-bit values) for MLPF_BF16 and MLPF_BF16_FP8FFN, as in a BF16
 * mixed-precision pre-LN block, whose embedding and residual branches all end in a bf16 product;
 * every residual sum is taken in FP32 and rounded once. */

/* Element embedding FFN (Sec. 5.3): h[T][d] = GELU(x W_e1 + b_e1) W_e2 + b_e2 for every row,
 * x[T][F] FP32. */
mlpf_status_t mlpf_embed(mlpf_model_t model, const float* x, const mlpf_batch_t* batch, void* h,
                         void* ws, size_t ws_bytes, void* stream);

/* The transformer encoder (Sec. 5.3, Eq. 4), in place on h [S][T][d]: S = 1 for
 * MLPF_TOPO_SERIAL, 2 for MLPF_TOPO_PARALLEL2. On entry h[0] holds the embedding; on return h[s]
 * holds stack s's output (h[1] is overwritten for PARALLEL2). */
mlpf_status_t mlpf_encoder_forward(mlpf_model_t model, void* h, const mlpf_batch_t* batch,
                                   void* ws, size_t ws_bytes, void* stream);

/* Output heads and the inference rule (Sec. 5.3, Eq. 2): from h ([S][T][d], as left by
 * mlpf_encoder_forward) writes logits[T][6], reg[T][5] (pT', eta, sin phi, cos phi, E'), and
 * cls[T] (int32), the class the config's decision rule takes from the six logits (ARGMAX: their
 * argmax; BINARY: 0 unless the binary logit is positive, else 1 + the particle-type argmax). If
 * prim (FP32 [T][2]: primary pT, E) and decoded (FP32 [T][4]) are both non-NULL, decoded gets
 * (pT, eta, phi, E). */
mlpf_status_t mlpf_heads(mlpf_model_t model, const void* h, const mlpf_batch_t* batch,
                         float* logits, float* reg, int32_t* cls, const float* prim,
                         float* decoded, void* ws, size_t ws_bytes, void* stream);

/* mlpf_embed + mlpf_encoder_forward + mlpf_heads with h inside the workspace: one event set in,
 * per-element outputs out. Graph-capturable (no allocation, no synchronisation, no memset). */
mlpf_status_t mlpf_reconstruct_events(mlpf_model_t model, const float* x,
                                      const mlpf_batch_t* batch, float* logits, float* reg,
                                      int32_t* cls, const float* prim, float* decoded, void* ws,
                                      size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, hosts that forbid allocation): mlpf_reconstruct_events without the workspace argument.
 * Its scratch is a fixed array of 128 MiB in device memory that the library holds on each GPU it
 * runs on from its load until the process ends; the call allocates nothing (no hipMalloc, no
 * library routine that allocates). Batches whose workspace (mlpf_workspace_bytes) exceeds 128 MiB
 * return MLPF_ERR_CAPACITY with nothing enqueued (a d_model 256 BF16 model fits about 20,000 rows,
 * e.g. two events of 8192 elements). Every call on one GPU uses the same scratch: calls that
 * overlap on a GPU (on different streams, or from different threads without ordering) race and
 * give wrong results; calls ordered on one stream are safe. Nothing in the scratch needs to start
 * at zero. Other arguments, errors and results as mlpf_reconstruct_events (bitwise the same). */
mlpf_status_t mlpf_reconstruct_events_noalloc(mlpf_model_t model, const float* x,
                                              const mlpf_batch_t* batch, float* logits, float* reg,
                                              int32_t* cls, const float* prim, float* decoded,
                                              void* stream);

/* Particle candidates per event (Sec. 5.3: at inference an element yields a particle when its
 * predicted class is a particle, with that class and the four-momentum of its heads; Sec. 8: the
 * reconstruction module turns the outputs into a list of candidates per event). From cls[T] (as
 * written by mlpf_heads; 0 = no particle) and optionally decoded[T][4] (pT, eta, phi, E), keeps
 * every valid element of every event with cls != 0, in element order within its event, events in
 * order. Writes event_offsets[n_events + 1] (device int32): event e's candidates are entries
 * event_offsets[e] .. event_offsets[e+1]-1, and event_offsets[n_events] is their total; for each
 * entry k < cap: cand_row[k] (device int32, the row of the element), cand_cls[k] (its class), and,
 * when cand_kin is non-NULL, cand_kin[k][4] = decoded[row] (cand_kin and decoded 16-byte aligned).
 * Entries k >= cap are not written: a total above cap means the list was cut (the caller sizes cap,
 * e.g. to total_rows, or reads the total and calls again). The batch description is clamped as
 * in the forward calls. Allocates nothing; three kernel launches on `stream`; graph-capturable.
 * MLPF_ERR_INVALID_ARG for NULL required pointers, negative sizes or misaligned kinematics. */
mlpf_status_t mlpf_candidates(const mlpf_batch_t* batch, const int32_t* cls, const float* decoded,
                              int32_t* event_offsets, int32_t* cand_row, int32_t* cand_cls,
                              float* cand_kin, int32_t cap, void* stream);

/* Captured forward passes (HIP graphs). mlpf_graph_create captures one mlpf_reconstruct_events
 * call with exactly these arguments on `stream` (which must not be the NULL stream; nothing is
 * executed during capture) and instantiates it. Every kernel reads the batch description
 * (row_start, n_valid) and the inputs from the given device buffers when the graph runs, and sizes
 * its launch from the host values of `batch`, which become capacities: a replay computes any batch
 * whose buffers are rewritten in place with at most batch->total_rows rows, batch->n_events events
 * (trailing unused events given zero rows by repeating the last row_start value) and valid counts
 * <= batch->max_seqlen. Rows beyond the last event cost nothing. The graph borrows all buffers and
 * the model. Launches of one graph must be serialised (they share the workspace). */
typedef struct mlpf_graph_s* mlpf_graph_t;
mlpf_status_t mlpf_graph_create(mlpf_model_t model, const float* x, const mlpf_batch_t* batch,
                                float* logits, float* reg, int32_t* cls, const float* prim,
                                float* decoded, void* ws, size_t ws_bytes, void* stream,
                                mlpf_graph_t* out);
mlpf_status_t mlpf_graph_launch(mlpf_graph_t graph, void* stream);
mlpf_status_t mlpf_graph_destroy(mlpf_graph_t graph);

/* Optional per-kernel timing for benchmarks. While enabled on a model, every launch of a kernel
 * class (below) made through that model is bracketed by a pair of HIP events recorded on the launch
 * stream (event objects are created on first use; do not enable it around graph capture).
 * mlpf_profiler_enable(model, 1) also resets the counters; mlpf_profiler_read returns the summed
 * event-to-event time and the launch count of one class since then, and needs every stream that
 * was used to have been synchronised (else MLPF_ERR_HIP "not ready"). Not thread-safe against
 * concurrent forward calls on the same model while enabled. */
typedef enum {
  MLPF_PROF_EMBED = 0,     /* both products of the embedding FFN */
  MLPF_PROF_QKV = 1,       /* LN1 + Q/K/V projection */
  MLPF_PROF_ATTENTION = 2, /* fused masked varlen attention */
  MLPF_PROF_OUTPROJ = 3,   /* attention output projection + residual (+ LN2 unless fused FFN) */
  MLPF_PROF_FFN1 = 4,      /* FFN1 + GELU (the whole fused FFN, LN2 included, when it runs) */
  MLPF_PROF_FFN2 = 5,      /* FFN2 + residual */
  MLPF_PROF_HEADS = 6,     /* both head layers, argmax, decode */
  MLPF_PROF_WORKLIST = 7,  /* batch sanitising and attention work list */
  MLPF_PROF_CLASSES = 8
} mlpf_prof_class_t;
mlpf_status_t mlpf_profiler_enable(mlpf_model_t model, int enable);
mlpf_status_t mlpf_profiler_read(mlpf_model_t model, int kernel_class, double* total_ms,
                                 int64_t* launches);

/* Launch-shape choices. Each product of the forward pass (mlpf_op_t) runs with one of a fixed set
 * of tile shapes; by default a size-based rule picks it per call. mlpf_tune_set pins op to tile
 * (0 <= tile < mlpf_tune_count(op)) or restores the rule (tile = -1); this is how the autotuner
 * stores its choice. Tile shapes change speed only: in BF16 and FP8 every GEMM tile sums k in the
 * same order, so GEMM results are bitwise identical across tiles; in FP32 the k-tile length sets
 * the grouping of the partial sums, so tiles with equal k-tile lengths agree bitwise and others to
 * rounding. Attention tiles change the order of the softmax sums (results differ by rounding
 * only). Not thread-safe against concurrent forward calls on the same model. */
typedef enum {
  MLPF_OP_EMBED1 = 0, MLPF_OP_EMBED2 = 1, MLPF_OP_QKV = 2, MLPF_OP_OUTPROJ = 3,
  MLPF_OP_FFN1 = 4, MLPF_OP_FFN2 = 5, MLPF_OP_HEADS1 = 6, MLPF_OP_ATTENTION = 7,
  /* How the feed-forward block runs: tile 0 = two products (FFN1 with GELU, FFN2 with the residual
   * update, tiles of MLPF_OP_FFN1/FFN2 apply); tiles 1 to 3 = one fused kernel that keeps the
   * d_ff-wide intermediate on chip (1: 128 rows per workgroup, double-buffered weights; 2: 64
   * rows, single-buffered, two workgroups per CU; 3: as 1, with persistent workgroups that loop
   * over the row tiles and overlap one tile's end with the next one's start, the default when d_ff
   * is not a multiple of 128; 4: as 3, software-pipelined: the GELU of one 64-unit chunk runs
   * beside the first product of the next, d_ff a multiple of 128 only, the default there), for
   * MLPF_BF16 models with d_model 64, 128 or 256, bitwise equal
   * to tile 0 with any GEMM tiles; tiles 5 to 8 (9 to 12) = the shape of 2 (of 1) with the hidden
   * units split into 2, 4, 8 or 16 equal parts (a divisor of d_ff / 64, else
   * MLPF_ERR_UNSUPPORTED), one workgroup per (row tile, part) writing its FP32 partial product to
   * the workspace, then a kernel that adds the parts in order, the bias and the residual (and the
   * next block's LN1): for launches too small to fill the chip; results differ from tile 0 by the
   * rounding of the partial sums. The part count is capped like the attention's key splits (8, 4
   * or 2 for up to 4096, 8192 or 16384 rows; beyond, tiles 5 to 12 run unsplit in their shape).
   * The rule (-1) splits when the rows fit under that cap, into the fewest parts that give two
   * 64-row workgroups per CU, else runs tile 4 (or 3). Setting 1 to 12 on another model returns
   * MLPF_ERR_UNSUPPORTED. FP8 calibration always runs the two products. */
  MLPF_OP_FFN = 8,
  /* How the output heads run: tile 0 = the first-layer product (tiles of MLPF_OP_HEADS1 apply)
   * writing the five GELU hidden layers, then a kernel for the second layer, argmax and decode;
   * tile 1 = the first-layer product with 64 x 256 tiles whose epilogue also takes the second
   * layer of its head (the hidden layer never leaves the chip), then a per-row kernel for the
   * biases, argmax and decode (the default; bf16 models with d_model 256 only, else
   * MLPF_ERR_UNSUPPORTED). The two differ by the order of the second-layer sums (rounding). */
  MLPF_OP_HEADS = 9,
  /* Key splits of the BF16 score-bound attention (kinds 1 and 2): tile t = 2^t splits (1, 2, 4,
   * 8). With s > 1 every work item runs as s workgroups, each over one contiguous range of the
   * event's keys, writing unnormalised partial outputs with their row sums and exponent offsets
   * to the workspace; a second kernel combines them exactly (O = sum_s 2^(m_s - M) O_s /
   * sum_s 2^(m_s - M) l_s). Results differ from one split by rounding. The rule (-1) splits only
   * launches too small to fill the chip (about three waves per SIMD when the rows form one
   * event), and never beyond 8, 4 or 2 splits for up to 4096, 8192 or 16384 rows (the
   * workspace's partial buffers; no split beyond 16384 rows); a pinned count is capped the same
   * way. FP32 models and kind 0 never split. */
  MLPF_OP_ATTN_SPLIT = 10,
  MLPF_OP_COUNT = 11
} mlpf_op_t;
int32_t mlpf_tune_count(int32_t op);
mlpf_status_t mlpf_tune_set(mlpf_model_t model, int32_t op, int32_t tile);
int32_t mlpf_tune_get(mlpf_model_t model, int32_t op); /* -1 = size-based rule */
/* Shape of tile `tile` of op, written to shape[6]: GEMM ops {rows, columns, wave rows, wave
 * columns, bytes per operand row and k-tile, schedule: one workgroup per tile (0), persistent (1), or
 * one workgroup per tile whose k-tiles travel by direct-to-LDS loads through three LDS stages (2;
 * products with an FP32 A operand that the kernel converts run such tiles' shape as 0)};
 * MLPF_OP_ATTENTION {waves per workgroup, keys per LDS stage, 32-query blocks per wave, kernel
 * kind (0: online softmax with running maxima, 1: BF16 score-bound offset, 2: the same without the
 * look-ahead QK^T product; FP32 runs kind 0),
 * 0, 0}; MLPF_OP_FFN {hidden-unit parts of one fused kernel (1: all at once, 2 to 16: split) or 0
 * for two products, rows per workgroup, waves, double buffered, persistent, pipelined};
 * MLPF_OP_HEADS {fused (1) or not (0), rows and columns of the fused tile, 0, 0, 0};
 * MLPF_OP_ATTN_SPLIT {splits, 0, 0, 0, 0, 0}. MLPF_ERR_INVALID_ARG for an op or tile out of range or a NULL shape. */
mlpf_status_t mlpf_tune_shape(int32_t op, int32_t tile, int32_t* shape);

/* FP8 activation calibration for MLPF_BF16_FP8FFN. Runs the embedding and encoder of `model` (an
 * FP32 or BF16 model) on the batch and raises amax[2l] to max |LN2 output| and amax[2l+1] to
 * max |act(FFN1)| of block l, over every live row (so calibration batches should carry no padding
 * rows). amax: device FP32 [2 n_layers] holding non-negative values on entry (zero it before the
 * first batch; calls accumulate the maximum). Its final values are the act_amax argument of
 * mlpf_model_create. */
mlpf_status_t mlpf_calibrate_fp8(mlpf_model_t model, const float* x, const mlpf_batch_t* batch,
                                 float* amax, void* ws, size_t ws_bytes, void* stream);

/* Masked variable-length multi-head self-attention alone (Eq. 4): for every event e and head j,
 *   o[rows of e][j*d_head .. (j+1)*d_head-1] = softmax(q_j k_j^T / sqrt(d_head)) v_j
 * where the keys are the event's valid rows only. q, k, v: [n_heads][total_rows][d_head]
 * (head-major), o: [total_rows][d_model], all in the operand type of the model's precision (FP32
 * for MLPF_FP32, BF16 otherwise); q is not pre-scaled. Rows beyond an event's valid count are not
 * written. Uses the same kernel as mlpf_encoder_forward (which computes q, k, v itself). */
mlpf_status_t mlpf_attention_forward(mlpf_model_t model, const void* q, const void* k,
                                     const void* v, void* o, const mlpf_batch_t* batch, void* ws,
                                     size_t ws_bytes, void* stream);

const char* mlpf_status_string(mlpf_status_t status);
const char* mlpf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MLPF_H */
