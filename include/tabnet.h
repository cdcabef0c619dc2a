/*
 * tabnet.h -- C ABI of libtabnet, batched TabNet inference on AMD Instinct MI355X (gfx950).
 *
 * What the library computes.  The paper deploys TabNet so that every invocation
 * returns predictions together with feature-attribution masks (Sec. III-B), the
 * masks being produced inside the forward pass by sparsemax (Sec. V-C); the model is
 * loaded into GPU memory once and reused across invocations of caller-chosen batch
 * size (Sec. III-B).  TabNet itself is the model the paper cites (Sec. I, Sec. II-B):
 * per decision step an attentive transformer scales its scores by a prior and
 * applies sparsemax to obtain the step mask M_i; the masked, batch-normalised input
 * goes through a feature transformer of GLU layers; the decision halves are summed
 * after ReLU into the output map, and the aggregate mask is sum_i eta_i M_i
 * normalised per row, with eta_i the row's total ReLU decision mass at step i.
 *
 * Conventions shared by every entry point
 *   - Functions return a tabnet_status; no C++ exception crosses this boundary.
 *     On a non-OK status tabnet_last_error() returns a message for the calling thread.
 *   - Matrices are dense, row-major, float32, with no padding between rows.
 *   - Device pointers are plain HIP device addresses on the handle's device; the
 *     caller owns them and keeps them alive until the work that uses them finishes.
 *   - Invalid arguments are rejected before any GPU work is enqueued.
 */
#ifndef TABNET_H
#define TABNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TABNET_OK = 0,
    TABNET_E_INVALID = -1,     /* bad argument or inconsistent model header            */
    TABNET_E_OOM = -2,         /* device or host allocation failed                     */
    TABNET_E_HIP = -3,         /* a HIP runtime call failed; the handle is now failed  */
    TABNET_E_IO = -4,          /* weight file missing, truncated, or bad magic/version */
    TABNET_E_ADMISSION = -5,   /* request larger than the server's memory budget       */
    TABNET_E_TIMEOUT = -6,     /* wait ended before the request completed              */
    TABNET_E_STOPPED = -7,     /* server stopped; request cancelled                    */
    TABNET_E_UNSUPPORTED = -8  /* model shape outside the compiled kernel set          */
} tabnet_status;

typedef enum {
    TABNET_FP32 = 0,      /* FP32 MFMA GEMMs, FP32 everything                            */
    TABNET_BF16 = 1,      /* BF16 GEMM operands (RNE), FP32 accumulate and epilogues      */
    TABNET_FP8_E4M3 = 2,  /* E4M3 weights and GEMM inputs, one scale per row; see below  */
    TABNET_INT8 = 3,      /* INT8 weights and GEMM inputs, INT32 products; see below      */
    TABNET_MXFP8 = 4,     /* OCP MX: E4M3 elements in blocks of 32 with E8M0 scales       */
    TABNET_MXFP4 = 5,     /* OCP MX: E2M1 elements in blocks of 32 with E8M0 scales       */
    TABNET_MXFP6 = 6,     /* OCP MX: E2M3 elements in blocks of 32 with E8M0 scales       */
    TABNET_MXFP8_E5M2 = 7,  /* OCP MX: E5M2 elements in blocks of 32 with E8M0 scales     */
    TABNET_MXFP6_E3M2 = 8,  /* OCP MX: E3M2 elements in blocks of 32 with E8M0 scales     */
    TABNET_FP8_WEIGHTS = 9  /* E4M3 weights, one scale per output channel; BF16 inputs    */
} tabnet_precision;

/* Model hyper-parameters as stored in the weight file.  N = n_d + n_a. */
typedef struct {
    int32_t D;          /* input features (columns of X)                               */
    int32_t n_d;        /* decision width                                              */
    int32_t n_a;        /* attention width                                             */
    int32_t n_steps;    /* decision steps S (masks per row)                            */
    int32_t n_shared;   /* GLU layers shared by every feature-transformer pass         */
    int32_t n_indep;    /* GLU layers owned by each pass                               */
    int32_t n_out;      /* output logits per row                                       */
    int32_t reserved;
    double gamma;       /* prior relaxation: P <- P * (gamma - M)                      */
    double bn_eps;      /* batch-norm epsilon                                          */
} tabnet_config;

typedef struct tabnet_handle tabnet_handle;

/*
 * tabnet_load -- read a TNW1 weight file, fold every inference batch norm into the
 * preceding linear map in FP64 (W' = diag(g / sqrt(v + eps)) W, b' = beta - s * mean;
 * the input batch norm becomes a per-column affine map), round the folded weights to
 * the requested precision, pack them in the MFMA operand order of the kernels and copy
 * them to `device`.  The model is then resident: the paper loads its model into GPU
 * memory once at cold start and reuses it (Sec. III-B).
 *
 *   path       TNW1 file (format: header of 64 bytes, then float32 parameters)
 *   precision  a tabnet_precision value
 *   device     HIP device ordinal
 *   out        receives the new handle; the caller releases it with tabnet_free
 *
 * Errors: TABNET_E_IO (missing / truncated / bad magic), TABNET_E_INVALID (header
 * fields out of range, e.g. n_d < 1 or gamma < 1), TABNET_E_UNSUPPORTED (no compiled
 * kernel covers D, n_d + n_a or n_out), TABNET_E_OOM, TABNET_E_HIP.
 *
 * Shapes.  Every precision has kernels compiled for the shape families of ceil(D / 16),
 * ceil((n_d + n_a) / 16) and floor(n_d / 16) = (1..4, 1, 0), (4, 2, 1), (7, 4, 2),
 * (13, 8, 4) and, on the split-feature kernel, (32, 8, 4) (D = 497..512).  Any other model
 * with D <= 512 and n_d + n_a <= 128 runs in TABNET_FP32, TABNET_BF16, TABNET_FP8_WEIGHTS,
 * TABNET_FP8_E4M3 and TABNET_INT8 on a generic kernel: up to D = 208 the register-resident one compiled for 4, 8 or 13 feature tiles
 * and 1, 2, 4 or 8 hidden tiles, past it the split-feature one compiled for 32 and 8 (the
 * padding is masked or carried as zeros); the other precisions refuse it.  Raw rows
 * (tabnet_set_embeddings) run on such a model in TABNET_FP32 and TABNET_BF16 up to D = 208
 * and are refused otherwise.
 *
 * TABNET_FP8_E4M3 puts both operands of every GEMM in E4M3 with one FP32 scale per
 * vector: each weight row as q = E4M3(W'_n / sigma_n) with sigma_n = max_k |W'_nk| / 448,
 * and each GEMM input row (coded in the kernel) as E4M3(u / s_r) with s_r = max_k |u_k| / 448,
 * both rounded to nearest even.  The FP8 matrix instruction sums the products in FP32,
 * dequantised by sigma_n * s_r before the folded shift is added; the GLU and residual
 * epilogues, the prior, sparsemax and aggregation stay in FP32.
 *
 * TABNET_FP8_WEIGHTS stores the weights as TABNET_FP8_E4M3 does (E4M3 codes, one scale
 * sigma_n per output channel) and keeps the GEMM inputs in BF16 (round to nearest even):
 * the codes are widened to BF16 in registers (exactly: every E4M3 value is a BF16 value),
 * the BF16 matrix instruction sums the products in FP32, and the sum is scaled by sigma_n
 * before the folded shift is added.  It halves the weight bytes of BF16 and leaves the
 * activations' precision as in TABNET_BF16.
 *
 * TABNET_INT8 is the paper's FP32-to-INT8 quantisation (Sec. VI-D) in symmetric form:
 * each GEMM weight row is stored as integer codes in [-127, 127] with one FP32 scale
 * sigma_n = max_k |W'_nk| / 127, and each GEMM input row (the masked features, the
 * hidden state, or its attention half for the attentive transformer) is coded the same
 * way on the fly, with its own step max_k |u_k| / 127 and ties rounded to even.  The
 * products are exact INT32 sums on the integer matrix cores, dequantised by
 * sigma_n * step before the folded shift is added; everything else stays in FP32.
 * A row that holds a non-finite value gets unspecified outputs (other rows are not
 * affected).  Both run on every compiled shape, the split-feature kernel (the 512-feature
 * shape) included: there every wave reads the whole GEMM input from LDS and takes the
 * row's scale itself.
 *
 * TABNET_MXFP8 / TABNET_MXFP8_E5M2 / TABNET_MXFP6 / TABNET_MXFP6_E3M2 / TABNET_MXFP4 put
 * both operands of every GEMM in an OCP microscaling format: along K, blocks of 32 values
 * share one power-of-two scale 2^X (E8M0) with X = floor(log2 max|v|) - emax (8 for
 * E4M3, 15 for E5M2, 2 for E2M3 and E2M1, 4 for E3M2), and each value is stored as
 * v / 2^X rounded to nearest even in the element format, saturating (+-448, +-57344,
 * +-7.5, +-28, +-6).  The
 * weights are coded at load, each GEMM input row in the kernel; the gfx950 scaled matrix
 * instruction applies both scales, and everything else stays in FP32.  A block is 32
 * consecutive K positions of the GEMM input in its own order (the attentive
 * transformer's input, the attention half, from its own first channel); a last block of
 * fewer positions holds the rest.  The kernel forms blocks from pairs of 16-channel
 * tiles, so a model whose attention half neither starts a tile (n_d % 16 == 0) nor fits
 * the tile pair it starts in (n_d % 16 + n_a <= 32) is TABNET_E_UNSUPPORTED in these
 * formats.  Non-finite behaviour as TABNET_INT8.  The split-feature kernel (the 512-feature
 * shape) has entries for all five MX forms; in the two 8-bit forms its weight slices leave
 * LDS for a final map of n_out x n_d <= 508 floats only (7 outputs at n_d = 64), and a
 * larger model is TABNET_E_UNSUPPORTED there.
 */
tabnet_status tabnet_load(const char* path, int precision, int device, tabnet_handle** out);

/* Copy the handle's model hyper-parameters to *out. */
tabnet_status tabnet_get_config(const tabnet_handle* h, tabnet_config* out);

/* Precision the handle was loaded with (a tabnet_precision value), or -1 for NULL. */
int tabnet_get_precision(const tabnet_handle* h);

/*
 * tabnet_forward -- batched TabNet inference, asynchronous on `stream`.
 *
 *   X           device, float32 [B, D]: raw feature rows (before the input batch norm)
 *   B           number of rows; 0 is valid and enqueues nothing
 *   logits      device, float32 [B, n_out]: W_fin * sum_i ReLU(d_i) per row
 *   masks_agg   device, float32 [B, D]: sum_i eta_i M_i divided by its row sum; a row
 *               whose sum is 0 is written as zeros
 *   masks_step  device, float32 [n_steps, B, D]: the sparsemax masks M_1..M_S; may be
 *               NULL, in which case the per-step masks are not written
 *   stream      hipStream_t to enqueue on; NULL means the device's null stream
 *
 * Every row is computed independently and in a fixed order, so a row's outputs do not
 * depend on the other rows of the batch or on B.  Errors: TABNET_E_INVALID (NULL
 * handle or required pointer, B < 0, B above 2^31 - 1), TABNET_E_HIP (launch failed;
 * the handle then refuses further work).  Overlapping calls on one handle from several
 * threads are not supported.
 */
tabnet_status tabnet_forward(tabnet_handle* h, const float* X, int64_t B, float* logits,
                             float* masks_agg, float* masks_step, void* stream);

/* ------------------------------------------------------------------------------------
 * Raw rows: categorical embedding in front of the model, masks per raw column.
 *
 * The paper's records reach the model after a preprocessing stage (Sec. III-A); the UCI
 * Adult rows carry 14 raw features (Sec. IV-A), and auditors read importance per raw
 * feature (Table IV) from the masks each invocation returns (Sec. III-B).  The model the
 * paper cites embeds every categorical column: level l of column c becomes row l of the
 * column's table, so C raw columns become D = sum_c dim_c model features (continuous
 * columns pass through).  The raw-row forward gathers the embeddings inside the fused
 * kernel (the D-wide rows never exist in memory) and writes each mask per raw column:
 * the sum of the column's model features.
 * ------------------------------------------------------------------------------------ */

/*
 * tabnet_set_embeddings -- attach a categorical embedding to a loaded model (replacing any
 * earlier one; waits for the device to be idle when it replaces one).
 *   n_cols   raw columns C, in order; the model features are the columns' widths laid end to end
 *   cards    host int32 [C]: levels of each categorical column; 0 marks a continuous column
 *   dims     host int32 [C]: embedding width of each column (1 for a continuous column);
 *            sum(dims) must equal the model's D
 *   tables   host float32: the categorical columns' tables, each [card, dim] row-major,
 *            concatenated in column order (copied; may be NULL if no column is categorical)
 * Errors: TABNET_E_INVALID (bad spec), TABNET_E_UNSUPPORTED, TABNET_E_OOM, TABNET_E_HIP.
 */
tabnet_status tabnet_set_embeddings(tabnet_handle* h, int32_t n_cols, const int32_t* cards, const int32_t* dims,
                                    const float* tables);

/*
 * tabnet_forward_raw -- tabnet_forward on raw rows, asynchronous on `stream`.
 *   X_raw            device, float32 [B, C]: continuous values, and in a categorical column the
 *                    level as a float (0, 1, ..., card - 1).  A value that is not such a level
 *                    (negative, too large, fractional, NaN) embeds as a zero vector.
 *   logits           device, float32 [B, n_out]
 *   masks_agg_cols   device, float32 [B, C]: the aggregate mask summed over each column's features
 *   masks_step_cols  device, float32 [n_steps, B, C] or NULL: each step mask, summed the same way
 * The logits equal those of tabnet_forward on the embedded rows bit for bit, and each column's
 * mask is the FP32 sum of that forward's masks over the column's features (formed on the
 * matrix cores as a product with the 0/1 feature-to-column map).
 * Errors: as tabnet_forward, and TABNET_E_INVALID if no embedding was set.
 */
tabnet_status tabnet_forward_raw(tabnet_handle* h, const float* X_raw, int64_t B, float* logits,
                                 float* masks_agg_cols, float* masks_step_cols, void* stream);

/* Release the device weights and the handle (NULL is ignored). Synchronises the device. */
void tabnet_free(tabnet_handle* h);

/* Message of the calling thread's last non-OK status ("" if none). Valid until the
 * thread's next call into the library. */
const char* tabnet_last_error(void);

/* Library ABI version (major * 100 + minor). */
int tabnet_abi_version(void);

/* ------------------------------------------------------------------------------------
 * Mask statistics.
 *
 * The paper assesses whether TabNet's explanations stay stable under production load by
 * the variance of each feature's mask value over many served rows, reported next to
 * each feature's importance (Sec. IV-C, Sec. V-C, Table IV).  These calls compute, on
 * the GPU, the per-feature mean (importance over a set of rows) and the population
 * variance of a mask matrix: for column d over the B rows,
 *     mean_d = (1/B) sum_r m[r][d],   var_d = (1/B) sum_r (m[r][d] - mean_d)^2.
 * Sums are taken in FP64 around the column's first value (shifted sums) and added in a
 * fixed order: the result is the same on every run.
 * ------------------------------------------------------------------------------------ */

/* Bytes of device workspace tabnet_mask_stats needs for B rows of D columns (0 if B < 1
 * or D < 1).  At most 1024 * 2 D * 8 bytes. */
size_t tabnet_mask_stats_workspace_bytes(int64_t B, int32_t D);

/*
 * tabnet_mask_stats -- per-column mean and population variance, asynchronous on `stream`.
 *
 *   masks       device, float32 [B, D] row-major: e.g. masks_agg, or one step of masks_step
 *   B, D        rows (>= 1) and columns (1 .. 2^24)
 *   mean, var   device, float64 [D] each: outputs
 *   workspace   device scratch of at least tabnet_mask_stats_workspace_bytes(B, D) bytes,
 *               caller-owned; it must not be used by other work until this call's work ends
 *   stream      hipStream_t on the calling thread's current device; NULL = null stream
 *
 * Errors: TABNET_E_INVALID (NULL pointer, B < 1, D out of range, workspace too small;
 * nothing is enqueued), TABNET_E_HIP (launch failed).
 */
tabnet_status tabnet_mask_stats(const float* masks, int64_t B, int32_t D, double* mean, double* var,
                                void* workspace, size_t workspace_bytes, void* stream);

/* Bytes of the library's own scratch for tabnet_mask_stats_noalloc (8 MiB per GPU). */
size_t tabnet_mask_stats_noalloc_max_bytes(void);

/*
 * tabnet_mask_stats_noalloc -- tabnet_mask_stats without a workspace argument, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same kernels, same results bit for bit.
 *
 *   masks, B, D, mean, var, stream   as in tabnet_mask_stats
 *
 * The partial sums live in a fixed device array of the library, one per GPU, held until
 * the process ends; the call allocates nothing.  Its first call on a device takes the
 * array's address on that device.  Every call on one GPU uses that GPU's array: calls
 * whose work overlaps on one GPU (other streams, other threads) race and must be
 * ordered by the caller.  Nothing in the array needs clearing between calls: each call
 * writes every partial sum it reads.
 *
 * Errors: TABNET_E_INVALID (NULL pointer, B < 1, D out of range, or
 * tabnet_mask_stats_workspace_bytes(B, D) larger than tabnet_mask_stats_noalloc_max_bytes();
 * nothing is enqueued), TABNET_E_HIP (address lookup or launch failed).
 */
tabnet_status tabnet_mask_stats_noalloc(const float* masks, int64_t B, int32_t D, double* mean, double* var,
                                        void* stream);

/* ------------------------------------------------------------------------------------
 * Serving: continuous batching of variable-row requests.
 *
 * The paper serves TabNet per invocation with a batch size chosen at invocation time
 * (Sec. III-B) and names dynamic batching as the next optimisation (Sec. VI-D).  The
 * server batches requests as they arrive: a scheduler thread admits queued requests in
 * arrival order while their bytes fit a memory budget, packs the rows of the admitted
 * requests (a request may be split across launches) into one of `slots` launch buffers,
 * and enqueues copy-in, the fused forward and copy-out on that slot's stream, so
 * launches overlap on the device while later requests are being admitted.  A completion
 * thread copies each finished slice to the caller's buffers.  Every row is computed by
 * the same kernel as tabnet_forward, so a request's results do not depend on what it was
 * batched with.
 * ------------------------------------------------------------------------------------ */
typedef struct tabnet_server tabnet_server;

typedef struct {
    uint64_t mem_budget_bytes;     /* bytes of admitted, unfinished requests; 0 -> 8 GiB      */
    int32_t max_rows_per_launch;   /* rows per launch buffer; 0 -> 65536                     */
    int32_t slots;                 /* launch buffers (launches in flight); 0 -> 3, max 8     */
    int32_t with_step_masks;       /* 1: requests may ask for masks_step                      */
    int32_t use_graph;             /* 1: each slot's launch is a captured HIP graph          */
    int32_t mask_stats_window;     /* > 0: keep masks_agg statistics over each model's last
                                      mask_stats_window launches (tabnet_serve_mask_stats)     */
    int32_t reserved[3];
} tabnet_serve_opts;

typedef struct {
    uint64_t submitted, admitted, completed, rejected, cancelled;
    uint64_t rows_completed, launches;
    double p50_us, p99_us, p999_us, max_us, mean_us;  /* completion - arrival              */
    double rows_per_s;             /* completed rows / (last completion - first arrival)     */
    double mean_rows_per_launch;
    uint64_t inflight_bytes, peak_inflight_bytes;
} tabnet_serve_stats;

/*
 * tabnet_serve_start -- start a server over n_models resident models (handles stay owned
 * by the caller and must outlive the server; they must all be on one device).
 * opts may be NULL for the defaults.  Errors: TABNET_E_INVALID, TABNET_E_OOM, TABNET_E_HIP.
 */
tabnet_status tabnet_serve_start(tabnet_handle* const* models, int n_models,
                                 const tabnet_serve_opts* opts, tabnet_server** out);

/*
 * tabnet_serve_submit -- enqueue a request of `rows` rows for model index `model`.
 *   X_host           host, float32 [rows, D]; read during the call (copied), may be reused after
 *   logits_host      host, float32 [rows, n_out]; written before the request completes
 *   masks_agg_host   host, float32 [rows, D]
 *   masks_step_host  host, float32 [n_steps, rows, D] or NULL (ignored unless the server was
 *                    started with with_step_masks)
 *   arrival_ns       arrival time on the steady clock (tabnet_serve_now_ns), or 0 for "now";
 *                    latency is measured from it
 *   req_id           receives the request id
 * Output buffers must stay valid until tabnet_serve_wait / poll reports completion.
 * Errors: TABNET_E_INVALID; TABNET_E_ADMISSION if the request alone exceeds the budget;
 * TABNET_E_STOPPED after tabnet_serve_stop.  Thread-safe.
 */
tabnet_status tabnet_serve_submit(tabnet_server* s, int model, const float* X_host, int64_t rows,
                                  float* logits_host, float* masks_agg_host, float* masks_step_host,
                                  int64_t arrival_ns, uint64_t* req_id);

/* Wait up to timeout_us (< 0: forever) for a request.  TABNET_OK once its outputs are
 * written (the id is then released), TABNET_E_TIMEOUT, TABNET_E_STOPPED if it was cancelled,
 * TABNET_E_HIP if its launch failed, TABNET_E_INVALID for an unknown id.  Thread-safe. */
tabnet_status tabnet_serve_wait(tabnet_server* s, uint64_t req_id, int64_t timeout_us);

/* Non-blocking: *done = 1 (and the id is released) once the request finished; the status
 * is what tabnet_serve_wait would return. */
tabnet_status tabnet_serve_poll(tabnet_server* s, uint64_t req_id, int* done);

/* Counters and latency percentiles since start or the last reset.  (The getter is not
 * named tabnet_serve_stats: in C that name is the statistics struct's.) */
tabnet_status tabnet_serve_get_stats(tabnet_server* s, tabnet_serve_stats* out);
/* The same for the requests of one model: submitted, admitted, completed, rejected,
 * rows_completed, the latency percentiles and rows_per_s (its completed rows over the span
 * from its first arrival to its last completion) count that model's requests only;
 * launches and mean_rows_per_launch count the launches that served it; the in-flight
 * byte counters are the server's.  TABNET_E_INVALID for a bad model index. */
tabnet_status tabnet_serve_get_model_stats(tabnet_server* s, int model, tabnet_serve_stats* out);
tabnet_status tabnet_serve_reset_stats(tabnet_server* s);

/*
 * tabnet_serve_mask_stats -- per-feature mean and population variance of masks_agg over the
 * rows of model `model`'s last mask_stats_window completed launches (since start or the last
 * tabnet_serve_reset_stats): the served-load view of the mask stability the paper measures
 * (Sec. IV-C, Sec. V-C).  Each launch's statistics are computed on the GPU right after its
 * forward (tabnet_mask_stats' kernels, on the slot's stream) and the launches of the window
 * are merged on the host in FP64, oldest first.
 *   mean_host, var_host  host, float64 [D] of that model; zeros while no launch completed
 *   rows                 receives the number of rows in the window (may be NULL)
 * Errors: TABNET_E_INVALID (bad model index, NULL output, or the server was started with
 * mask_stats_window = 0).  Thread-safe.
 */
tabnet_status tabnet_serve_mask_stats(tabnet_server* s, int model, double* mean_host, double* var_host,
                                      int64_t* rows);

/* Steady-clock time in nanoseconds (the clock of arrival_ns). */
int64_t tabnet_serve_now_ns(void);

/* Stop admitting, cancel queued requests (they report TABNET_E_STOPPED), finish the
 * launches in flight, join the threads and free the server. */
tabnet_status tabnet_serve_stop(tabnet_server* s);

#ifdef __cplusplus
}
#endif
#endif /* TABNET_H */
