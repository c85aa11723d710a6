/*
 * xcorr.h -- C ABI of the MI355X (gfx950) X-stage library, libxcorr.so.
 *
 * The X-stage of an FX correlator (Sec. 1, Sec. 2.4 of Kocz et al., "A
 * Scalable Hybrid FPGA/GPU FX Correlator"): for every frequency channel c,
 * accumulate over an integration window the outer product of the vector of
 * channelised voltages of all inputs with its own conjugate,
 *
 *     V[c][i][j] = sum_t  x_i[c,t] * conj(x_j[c,t]),        0 <= j <= i < N_i,
 *
 * i.e. the lower triangle of x x^H including the autocorrelations (Sec. 2.4,
 * output-size equation), integrated on the GPU before it returns to the host
 * (Sec. 2.1, Sec. 4).  Inputs are twice the number of antennas, one per
 * polarisation (Sec. 2.2): input index i = 2 * antenna + pol.
 *
 * Data layout (all device memory, caller-owned, contiguous):
 *   input   [n_channels][n_time][n_inputs] samples
 *           XCORR_CI4: 1 byte per sample; high nibble = real part, low nibble =
 *                      imaginary part, both two's-complement 4-bit integers in
 *                      [-8, 7] (the 4+4-bit samples of Sec. 2.3).
 *           XCORR_CI8: 2 bytes per sample, int8 real then int8 imaginary (the
 *                      8-bit form of Sec. 2.4), full range [-128, 127].
 *   output  [n_channels][n_inputs*(n_inputs+1)/2][2], entry (i, j) at packed
 *           index i*(i+1)/2 + j, pair = (re, im).
 *           XCORR_PATH_I8_MFMA: int64 (exact sums).
 *           XCORR_PATH_F16_MFMA, XCORR_PATH_F32: float (fp32 accumulation).
 * The dump returns sums; the paper's time average is sum / samples_accumulated.
 *
 * Ownership and ordering: a plan owns its device accumulators until
 * xcorr_destroy.  Every call is enqueued on the plan's stream and returns
 * without waiting (except where noted); the caller must keep `d_in` unchanged
 * until the stream has passed the call, and `d_out` is valid once the stream
 * has passed the dump.  A plan is not thread-safe; distinct plans may be used
 * from distinct threads.
 *
 * Errors: every entry point returns an xcorr_status.  On any error nothing is
 * enqueued and the plan is unchanged; xcorr_last_error() gives a message
 * (thread-local).  No entry point throws or aborts.
 */
#ifndef XCORR_H
#define XCORR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    XCORR_OK = 0,
    XCORR_ERR_ARG = -1,          /* null/misaligned pointer, bad size or enum        */
    XCORR_ERR_NOMEM = -2,        /* device allocation failed                          */
    XCORR_ERR_DEVICE = -3,       /* HIP runtime error (see xcorr_last_error)          */
    XCORR_ERR_STATE = -4,        /* plan handle not valid                             */
    XCORR_ERR_UNSUPPORTED = -6   /* device is not gfx950, or shape not supported      */
} xcorr_status;

typedef enum { XCORR_CI4 = 0, XCORR_CI8 = 1 } xcorr_format;

typedef enum {
    XCORR_PATH_I8_MFMA = 0,      /* int8 MFMA, int32 partials, int64 output: exact    */
    XCORR_PATH_F16_MFMA = 1,     /* fp16 MFMA, fp32 accumulation, float output         */
    XCORR_PATH_F32 = 2           /* plain fp32 vector kernel, float output             */
} xcorr_path;

/* Plan flags. */
#define XCORR_FLAG_NO_XCD_MAP 0x2u /* dispatch work items in plain order (for tests)  */
#define XCORR_FLAG_OUT_I32 0x8u   /* int8 path: int32 (re, im) output; see below     */
#define XCORR_FLAG_NO_PERSIST 0x4u /* one workgroup per work item instead of the
                                      persistent schedule (LDS-DMA tiles; for tests)  */
/* XCORR_FLAG_OUT_I32: the int8 path writes each visibility as two int32
 * (re, im) instead of two int64 (8 bytes per baseline, as a complex float
 * would take).  Exact for any window of at most fold_bound samples between
 * resets, for both formats (the largest CI8 sums stay below 2^31); a call
 * that would take a window past fold_bound fails with XCORR_ERR_ARG and
 * changes nothing.  Not with the fp paths. */

/* Input counts: the kernels read rows of a multiple of 4 inputs (4-bit
 * samples) or 2 (8-bit), and the LDS-DMA tiles rows of a multiple of 16.
 * A plan whose n_inputs is not such a multiple first copies each chunk of
 * the caller's input, zero padded to that width, into a staging buffer it
 * holds and grows to its largest chunk (one extra pass over the input;
 * zero inputs add nothing, so results are unchanged).  The default tile
 * pads to 16 from 160 inputs up, where the window is bound by the matrix
 * cores; below that, rows that are a multiple of 4 (2) are read as they
 * are by the register tile.  Growing the buffer waits for the plan's
 * stream and allocates; xcorr_plan_bytes does not count it. */

/* Tile variants of the int8 path (xcorr_plan_desc.tile).  All give identical
 * (exact) results; they differ in how samples reach LDS. */
/* The LDS-DMA tiles copy rows as they are, 4-bit and 8-bit samples alike,
 * and transpose them in LDS reads; single plans and batches use them.
 * DMA8 takes 4-bit samples only. */
#define XCORR_TILE_DEFAULT 0       /* LDS-DMA depth 4 where allowed, else registers */
#define XCORR_TILE_DMA8 1          /* buffer loads straight to LDS, 8 steps in flight */
#define XCORR_TILE_DMA4 2          /* the same, 4 steps in flight                   */
#define XCORR_TILE_REGS 3          /* loads to registers, byte transposes, LDS writes */

typedef struct xcorr_plan_s* xcorr_plan_t;

typedef struct {
    int32_t n_inputs;            /* N_i, 1 .. 32768 (any count; see below)            */
    int32_t n_channels;          /* N_c >= 1                                          */
    int32_t format;              /* xcorr_format                                      */
    int32_t path;                /* xcorr_path                                        */
    void* stream;                /* hipStream_t, NULL = the null stream               */
    uint32_t flags;              /* XCORR_FLAG_*                                      */
    int32_t tile;                /* XCORR_TILE_*; 0 = default                         */
} xcorr_plan_desc;

typedef struct {
    int64_t samples_accumulated; /* samples summed into the dumped result            */
    int64_t start_sample;        /* running sample index at which this window began  */
    int64_t n_dumps;             /* dumps taken from this plan so far (incl. this)   */
} xcorr_dump_info;

typedef struct {
    size_t device_bytes;         /* device memory the plan holds                      */
    size_t output_bytes;         /* bytes of one dump                                 */
    size_t input_bytes_per_sample; /* bytes of one time sample of all channels       */
    int64_t fold_bound;          /* max samples per kernel launch (int32 partials)    */
    int32_t tile;                /* tile variant in use                               */
    int32_t work_items;          /* workgroups per launch (one time chunk)            */
    int32_t items_per_group;     /* workgroups per channel group                      */
    int32_t channels_per_group;  /* channels sharing one set of work items            */
} xcorr_plan_info;

/* Create a plan: validates the descriptor, checks the device is gfx950 and
 * allocates the plan's accumulators on the current device.  *out is set only
 * on success. */
xcorr_status xcorr_plan(xcorr_plan_t* out, const xcorr_plan_desc* desc);

/* Add n_time samples of every channel of d_in to the plan's accumulators.
 * d_in: device pointer, layout above, 16-byte aligned.  n_time == 0 is a
 * no-op.  Windows longer than fold_bound are split into several launches. */
xcorr_status xcorr_accumulate(xcorr_plan_t plan, const void* d_in, int64_t n_time);

/* Write the accumulated visibilities to d_out (device, layout above, 16-byte
 * aligned).  reset != 0 restarts the integration.  info may be NULL. */
xcorr_status xcorr_dump(xcorr_plan_t plan, void* d_out, int reset, xcorr_dump_info* info);

/* xcorr_accumulate followed by xcorr_dump, fused: the last launch writes the
 * result straight to d_out, so a window that starts from a reset plan costs
 * one read of the input and one write of the output. */
xcorr_status xcorr_accumulate_dump(xcorr_plan_t plan, const void* d_in, int64_t n_time,
                                   void* d_out, int reset, xcorr_dump_info* info);

/* Baseline-dependent integration (Sec. 5): dump only the baselines of the
 * selected 64 x 64 input-block tiles and, if reset != 0, restart their
 * integration, while the others keep integrating.  tile_select is a HOST
 * array of nr (nr + 1) / 2 bytes, nr = ceil(n_inputs / 64), in lower-triangle
 * tile order: tile (ti, tj), ti >= tj, at ti (ti + 1) / 2 + tj; nonzero =
 * selected.  Entries of d_out outside the selected tiles are left unchanged;
 * info->samples_accumulated counts samples since the plan's last full reset
 * (the per-tile count is the caller's cadence). */
xcorr_status xcorr_dump_tiles(xcorr_plan_t plan, void* d_out, const uint8_t* tile_select, int reset,
                              xcorr_dump_info* info);

/* Pulsar gating (Sec. 5): sample t of the window d_in (n_time samples,
 * layout of xcorr_accumulate) is integrated into plans[gate[t]]; gate is a
 * HOST array of n_time bytes, each < n_gates or 0xFF (sample discarded).
 * The plans (1..64, distinct) must share n_inputs, n_channels, format and
 * stream; their paths may differ.  Each gate's sample indices go to the
 * device (a list the first plan holds).  When every plan is an int8 plan
 * whose persistent depth-4 LDS-DMA launches read the caller's rows as they
 * are (n_inputs a multiple of 16, default or DMA4 tile, no
 * XCORR_FLAG_NO_PERSIST, channels below 2^31 bytes), each gate runs as its
 * plan's own launches (up to 8192 4-bit or 4096 8-bit samples each) that
 * copy the listed rows straight from d_in; otherwise the samples of each
 * gate are first packed together (one HBM pass over the kept samples, into
 * a buffer the first plan holds and grows as needed: up to the window's
 * size) and each gate runs over its packed rows.  Waits for the plans'
 * stream before the first launch (the sample lists are host temporaries).
 * Dump each gate's plan with xcorr_dump. */
xcorr_status xcorr_accumulate_gated(const xcorr_plan_t* plans, int32_t n_gates, const void* d_in, int64_t n_time,
                                    const uint8_t* gate);

/* Sizes and the work decomposition chosen for the plan. */
xcorr_status xcorr_query(xcorr_plan_t plan, xcorr_plan_info* info);

/* Bytes of device memory a plan with this descriptor would hold (admission
 * control); no allocation. */
xcorr_status xcorr_plan_bytes(const xcorr_plan_desc* desc, size_t* bytes);

/* Release the plan (waits for its stream).  Destroying NULL is XCORR_ERR_STATE. */
xcorr_status xcorr_destroy(xcorr_plan_t plan);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * integration window, the same result as xcorr_plan + xcorr_accumulate_dump
 * (reset) + xcorr_destroy with this descriptor, and the same kernels, but
 * no plan and no allocation.  The state those kernels need besides the
 * input and output -- the work-queue counters of the persistent launch and
 * the work-item table -- lives in a 4 MiB array inside the library, one per
 * GPU, kept until the process ends (its address is looked up once per
 * device, on the first call with that device current).
 *   desc   path XCORR_PATH_I8_MFMA, tile XCORR_TILE_DEFAULT; flags
 *          XCORR_FLAG_OUT_I32 / NO_XCD_MAP / NO_PERSIST as for a plan; work
 *          is enqueued on desc->stream.  n_inputs a multiple of 4 (CI4) or
 *          2 (CI8), up to the input count whose work-item table fits the
 *          array (87,376 items; every count up to 32768 fits).
 *   d_in   device, [n_channels][n_time][n_inputs] as for xcorr_accumulate
 *   d_out  device, [n_channels][n_inputs(n_inputs+1)/2][2], int64 (int32
 *          with XCORR_FLAG_OUT_I32), written completely
 * n_time must lie in [1, fold_bound] (one launch): longer windows need the
 * plan's accumulator, and are refused with XCORR_ERR_ARG.  Rows of a
 * multiple of 16 inputs take the LDS-DMA tile, others the register tile.
 * Each call clears the counters (a fill kernel) and copies the table (a
 * host-to-device copy of a table the library keeps for the process) before
 * its kernel, all on desc->stream; no hipMalloc, hipFree or other
 * allocating call is made.  Calls that overlap on one GPU share the array
 * and race: order them on one stream or synchronise between them. */
xcorr_status xcorr_correlate_noalloc(const xcorr_plan_desc* desc, const void* d_in, int64_t n_time, void* d_out);

/* ------------------------------------------------------------------------
 * Corner turn (Sec. 2.4): the X-stage input of a GPU assembled from captured
 * F-engine packets.  Capture places each packet by its sequence number
 * (block) and F-engine; a packet carries, for its spectra_per_packet
 * consecutive spectra one after another, every channel's inputs of that
 * F-engine (packet-format figure).  Completing the corner turn puts the
 * inputs of all F-engines of one channel and time next to each other; the
 * paper's unpacker also pads 4-bit samples to 8 bits (out_format XCORR_CI8).
 *
 *   d_packets  device, uint8 [n_blocks][n_fengines][S][n_channels][J],
 *              one 4+4-bit sample per byte, 16-byte aligned
 *   d_valid    device, uint8 [n_blocks][n_fengines], 0 = packet lost (its
 *              samples become zeros); NULL = all received
 *   d_out      device, [n_channels][n_blocks*S][n_fengines*J] bytes
 *              (XCORR_CI4) or [...][2] int8 (XCORR_CI8), 16-byte aligned:
 *              time = block * S + s, input = f * J + j
 * J = inputs_per_feng must be a multiple of 4; n_fengines * J <= 32768.
 * Enqueued on `stream`; nothing is allocated.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_blocks;            /* packets per F-engine in the buffer (sequence numbers) */
    int32_t n_fengines;          /* F-engines (FPGA nodes)                              */
    int32_t inputs_per_feng;     /* J, inputs per F-engine                              */
    int32_t n_channels;          /* channels of this GPU                                */
    int32_t spectra_per_packet;  /* S, consecutive spectra per packet                   */
} xcorr_packet_layout;

xcorr_status xcorr_corner_turn(const void* d_packets, const uint8_t* d_valid, const xcorr_packet_layout* layout,
                               int32_t out_format, void* d_out, void* stream);

/* ------------------------------------------------------------------------
 * F-stage (Sec. 2.3; Sec. 4: 8-bit real ADC samples at 200 MHz, a 2-tap
 * 8192-point polyphase filter bank, equalisation, 4+4-bit requantisation and
 * a contiguous run of channels), producing the X-stage input directly.
 *
 * For input a and spectrum m (N = n_points, P = n_taps):
 *   y[j]  = sum_{p<P} coeff[p N + j] * adc[a][(m + p) N + j],   j < N
 *   X[k]  = sum_j y[j] e^{-2 pi i j k / N},   channels k < N / 2
 *   v     = gain[a][k - chan_begin] * X[k]   for the kept channels
 *   CI4:  each component rounded half to even, saturated to [-7, 7], packed
 *         high nibble = real, low nibble = imaginary (two's complement)
 * n_spectra = n_samples / N - P + 1 (none if below 1); a stream continues
 * across calls when the caller keeps the last (P - 1) N samples in front.
 *
 *   d_adc      device, int8 [n_inputs][adc_stride], first n_samples used;
 *              adc_stride even
 *   d_coeff    device, float [P * N] prototype filter
 *   d_gain     device, float [n_inputs][n_chan]
 *   d_out      device; XCORR_FSTAGE_CI4: uint8 [n_chan][n_spectra][n_inputs],
 *              the layout xcorr_accumulate reads;
 *              XCORR_FSTAGE_F32: float [n_chan][n_spectra][n_inputs][2], the
 *              equalised values before requantisation
 *   d_work     device scratch of xcorr_fstage_work_bytes bytes (CI4 output:
 *              the codes in input-major order before the transpose into
 *              X-stage order); may be NULL for F32.  Caller-owned, contents
 *              undefined afterwards; calls that share it must not overlap.
 *   n_spectra  host, optional: receives n_spectra
 * Device pointers 16-byte aligned.  N must be 8192 and P 1 or 2
 * (XCORR_ERR_UNSUPPORTED otherwise).  fp32 arithmetic.  Enqueued on
 * `stream`; no device memory is allocated.  With CI4 output and at least
 * 1024 spectra the spectra go in 8 chunks, and the transpose of each chunk
 * runs on a second stream, after that chunk's transform and beside the next
 * one; the call returns with all its work ordered on `stream`.  The library
 * keeps one such stream (with its events) per device and caller stream,
 * created on first use; past 16 caller streams on a device the chunks of a
 * call run in order on `stream`.
 * ------------------------------------------------------------------------ */
#define XCORR_FSTAGE_CI4 0
#define XCORR_FSTAGE_F32 1

typedef struct {
    int32_t n_inputs;    /* ADC streams                                 */
    int32_t n_points;    /* N, transform length (8192)                  */
    int32_t n_taps;      /* P, filter-bank taps (1 or 2)                */
    int32_t chan_begin;  /* first kept channel                          */
    int32_t n_chan;      /* kept channels, chan_begin + n_chan <= N / 2 */
    int32_t out_kind;    /* XCORR_FSTAGE_CI4 or XCORR_FSTAGE_F32        */
} xcorr_fstage_desc;

xcorr_status xcorr_fstage(const xcorr_fstage_desc* desc, const void* d_adc, int64_t adc_stride, int64_t n_samples,
                          const float* d_coeff, const float* d_gain, void* d_work, void* d_out, int64_t* n_spectra,
                          void* stream);

/* Bytes of d_work that xcorr_fstage needs for this descriptor and sample
 * count (0 for F32 output). */
xcorr_status xcorr_fstage_work_bytes(const xcorr_fstage_desc* desc, int64_t n_samples, size_t* bytes);

/* ------------------------------------------------------------------------
 * Measurement support (not part of the method): the shader clock a kernel
 * runs at, which sets the MFMA peak it can reach (the int8 peak is 8192
 * ops per CU per cycle, so 5.03 POP/s at the 2.4 GHz peak clock of 256 CUs).
 * ------------------------------------------------------------------------ */

/* Launch one wave on `stream` (a hipStream_t, NULL = default stream) that
 * waits `ticks` ticks of the constant-rate wall clock (at most 2^22 polls,
 * so it always ends) and writes d_out[0..3] = wall-clock ticks at start and
 * end, shader cycles at start and end (uint64, device memory, 8-byte
 * aligned, caller-owned).  Launched on another stream beside a long kernel,
 * (d_out[3] - d_out[2]) / (d_out[1] - d_out[0]) * wall_khz is the shader
 * clock in kHz under that kernel's load.  *wall_khz receives the wall-clock
 * rate (host pointer; may be NULL).  Errors: XCORR_ERR_ARG for a null or
 * misaligned d_out or ticks outside [1, 2^32); XCORR_ERR_DEVICE if the
 * launch fails.  Nothing is enqueued on error. */
xcorr_status xcorr_clock_probe(void* d_out, int64_t ticks, int32_t* wall_khz, void* stream);

/* ------------------------------------------------------------------------
 * Batches: several plans (subarrays of uneven input and channel counts, the
 * X-stage of several arrays sharing one GPU, Sec. 3) run as ONE persistent
 * launch per time chunk.  Every plan of a batch must use XCORR_PATH_I8_MFMA
 * and the same format.  The batch borrows the plans: they must outlive it,
 * and while the batch is in use they must not be used on their own streams.
 * ------------------------------------------------------------------------ */
typedef struct xcorr_batch_s* xcorr_batch_t;

typedef struct {
    int32_t tile;                /* XCORR_TILE_* used for every plan of the batch    */
    int32_t grid;                /* persistent workgroups (multiple of 8)            */
    int32_t balance;             /* 1: XCD slices of equal cost; 0: equal item counts */
    int32_t reserved;
} xcorr_batch_config;

/* Create a batch over n_plans (1..64) plans; work is enqueued on `stream`
 * (hipStream_t, NULL = null stream).  Starts from the default configuration. */
xcorr_status xcorr_batch_create(xcorr_batch_t* out, const xcorr_plan_t* plans, int32_t n_plans,
                                void* stream);

/* One step for every plan k of the batch, in one launch per time chunk:
 * n_time[k] samples of d_in[k] (layout of xcorr_accumulate) are added to plan
 * k's integration; if d_out[k] is non-NULL the plan is then dumped to d_out[k]
 * (layout of xcorr_dump), restarting the integration if reset[k] != 0.
 * n_time[k] == 0 with d_out[k] == NULL leaves plan k untouched.  reset and
 * info may be NULL (no reset; no info); info[k] is filled for dumped plans. */
xcorr_status xcorr_batch_run(xcorr_batch_t batch, const void* const* d_in, const int64_t* n_time,
                             void* const* d_out, const int32_t* reset, xcorr_dump_info* info);

xcorr_status xcorr_batch_get_config(xcorr_batch_t batch, xcorr_batch_config* config);
xcorr_status xcorr_batch_set_config(xcorr_batch_t batch, const xcorr_batch_config* config);

/* Autotuner: times every candidate configuration (tile x grid x balance) on
 * `reps` windows of the given inputs (every plan must be freshly reset; the
 * windows are not kept) and keeps the fastest.  chosen and ms_best may be
 * NULL.  Synchronises the batch stream. */
xcorr_status xcorr_batch_autotune(xcorr_batch_t batch, const void* const* d_in, const int64_t* n_time,
                                  int32_t reps, xcorr_batch_config* chosen, float* ms_best);

/* Graphs: capture one integration step of the batch -- every plan k takes
 * n_time[k] > 0 samples from d_in[k] and is dumped with reset to d_out[k] --
 * as a hipGraph, and replay it.  Pointers and sizes are fixed at capture;
 * each replay is one full window per plan (plans must be freshly reset at
 * capture time and used only through the graph while it exists). */
typedef struct xcorr_graph_s* xcorr_graph_t;
xcorr_status xcorr_batch_capture(xcorr_batch_t batch, const void* const* d_in, const int64_t* n_time,
                                 void* const* d_out, xcorr_graph_t* graph);
xcorr_status xcorr_graph_launch(xcorr_graph_t graph);
xcorr_status xcorr_graph_destroy(xcorr_graph_t graph);

/* Release the batch (waits for its stream); the plans stay valid. */
xcorr_status xcorr_batch_destroy(xcorr_batch_t batch);

/* ------------------------------------------------------------------------
 * Server: a streaming loop over many integration streams (one stream = the
 * X-stage of one (sub)array, windows arriving over time, Sec. 2.1 / Sec. 4).
 *   - Streams are admitted by device memory: a stream needs the bytes of a
 *     plan of its descriptor (xcorr_plan_bytes); it is admitted when a slot
 *     and that much of the budget are free, else it waits (FIFO) and is
 *     admitted when closed streams release theirs.
 *   - A worker thread batches continuously: every launch takes windows
 *     that have arrived, of every admitted stream (windows that arrive while
 *     others are on the GPU join the next launch; up to 96 per launch,
 *     earliest deadline first (xcorr_server_set_deadline), each stream's in
 *     its own order; a window longer than fold_bound samples, or of a stream
 *     whose rows are staged zero padded, takes its stream's place in a
 *     launch alone), and runs them as one persistent launch per format
 *     group; up to max_inflight launches are queued on the server's stream.
 *   - Launch configurations are tuned online: for each mix (format group and
 *     the shapes of the admitted streams in it) every candidate (LDS-DMA
 *     depth or register tile, 1 or 2 workgroups per CU, slices of equal cost
 *     or equal item counts) runs 3 launches timed with events, and the one
 *     with the most complex MACs per second of launch time is kept.  With
 *     tune_path set, kept configurations are appended to that text file
 *     (one "mix tile grid balance" line each) and read back when a server is
 *     created, so a known mix starts tuned.
 *   - Each window is accumulated and dumped with reset (one integration per
 *     window); the caller keeps d_in and d_out valid until its ticket is done.
 * Results do not depend on what else is in the batch (exact int8 path).
 * ------------------------------------------------------------------------ */
typedef struct xcorr_server_s* xcorr_server_t;

typedef struct {
    size_t device_budget;        /* bytes of plan memory the server may hold        */
    int32_t max_streams;         /* admitted streams at once (1..64)                */
    int32_t max_inflight;        /* launches queued on the stream at once (1..8)    */
    void* stream;                /* hipStream_t for all work; NULL = null stream    */
    const char* tune_path;       /* launch-configuration cache file, or NULL        */
} xcorr_server_desc;

typedef struct {
    int64_t windows_done;        /* windows whose dump is complete                  */
    int64_t launches;            /* batched launches issued                         */
    double cmac;                 /* complex MACs of the completed windows           */
    double elapsed_s;            /* first submit to last completion                 */
    double latency_p50_ms;       /* submit -> dump complete, over completed windows */
    double latency_p99_ms;
    double latency_max_ms;
    double mean_batch;           /* windows per launch                              */
    int32_t streams_admitted;    /* currently admitted                              */
    int32_t streams_waiting;     /* opened, waiting for memory or a slot            */
    size_t device_bytes;         /* plan memory held now                            */
    int32_t mixes_tuned;         /* mixes whose launch configuration is settled     */
    int32_t mixes_tuning;        /* mixes whose candidates are still being timed    */
    int64_t deadline_misses;     /* completed windows that finished past their deadline */
} xcorr_server_stats;

/* Create a server and start its worker thread (on the current device). */
xcorr_status xcorr_server_create(xcorr_server_t* out, const xcorr_server_desc* desc);

/* Open a stream with the plan descriptor desc (path must be
 * XCORR_PATH_I8_MFMA; desc->stream is ignored).  *stream_id is set at once;
 * admission happens now or later.  XCORR_ERR_NOMEM if the stream could never
 * fit the budget. */
xcorr_status xcorr_server_open(xcorr_server_t server, const xcorr_plan_desc* desc, int32_t* stream_id);

/* Queue one window of n_time > 0 samples (device buffer d_in, layout of
 * xcorr_accumulate) whose dump goes to d_out (layout of xcorr_dump).  The
 * caller must have ordered the writes of d_in before this call (e.g. by
 * synchronising the stream that produced it).  *ticket identifies it. */
xcorr_status xcorr_server_submit(xcorr_server_t server, int32_t stream_id, const void* d_in, int64_t n_time,
                                 void* d_out, int64_t* ticket);

/* done = 1 once the window's dump is complete in d_out; then info (may be
 * NULL) and latency_ms (submit -> completion, may be NULL) are filled.
 * xcorr_server_wait blocks until done. */
xcorr_status xcorr_server_poll(xcorr_server_t server, int64_t ticket, int32_t* done, xcorr_dump_info* info,
                               double* latency_ms);
xcorr_status xcorr_server_wait(xcorr_server_t server, int64_t ticket, xcorr_dump_info* info, double* latency_ms);

/* Real-time deadlines (Sec. 3: a correlator keeps up when each window is
 * done before the next one has arrived): from now on a window of n_time
 * samples submitted to this stream is due n_time * sample_period_s seconds
 * after its submission (0 = no deadline, the default).  The worker orders
 * pending windows by deadline and closes a launch before it would make a
 * window in it late that could still be on time (a throughput model of
 * recent launches estimates their time), so that short urgent windows do
 * not wait behind long ones; when the most urgent window is late anyway,
 * the launch may take twice its time (at least 0.25 ms) of later windows
 * to catch up.  Windows without a deadline come last.  Misses are counted
 * in the stats. */
xcorr_status xcorr_server_set_deadline(xcorr_server_t server, int32_t stream_id, double sample_period_s);

/* Close a stream: no more submits; its plan memory is released once its
 * queued windows are done, which may admit waiting streams. */
xcorr_status xcorr_server_close(xcorr_server_t server, int32_t stream_id);

xcorr_status xcorr_server_query(xcorr_server_t server, xcorr_server_stats* stats);

/* Finish every queued window, stop the worker and release everything. */
xcorr_status xcorr_server_destroy(xcorr_server_t server);

const char* xcorr_strerror(xcorr_status status);
const char* xcorr_last_error(void);

/* Library version, 10000 * major + 100 * minor + patch. */
int32_t xcorr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* XCORR_H */
