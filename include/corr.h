/*
 * corr.h -- C ABI of libcorr, an FX correlator for AMD MI355X (gfx950).
 *
 * The operations follow Wayth, Greenhill & Briggs (2009), "A GPU based
 * real-time software correlation system for the Murchison Widefield Array
 * prototype" (arXiv:0906.1887):
 *   - configure N_I inputs and N_C channels (Sec. 4, opening);
 *   - channelise each input's real sample blocks with an FFT, 2 N_C samples to
 *     N_C channels with the redundant half dropped (Sec. 2, Sec. 4 "second step");
 *   - cross-multiply every spectrum with the conjugate of every other and
 *     accumulate, all N_I(N_I+1)/2 products incl. autos (Sec. 2, Sec. 4
 *     "third step", Fig. 2);
 *   - read the accumulators with their update count and reset them (Fig. 1).
 *
 * Conventions
 *   Visibility   V_ij[c] = sum_t x_i[c,t] * conj(x_j[c,t]).
 *   Output       [n_channels][P][2] (re, im), P = N_I(N_I+1)/2, packed lower
 *                triangle, row-major: b(i,j) = i(i+1)/2 + j for 0 <= j <= i.
 *                Element type: int32 for CORR_X_I8, float32 for the other
 *                engines, float64 for the long-run accumulator.  Im of every
 *                auto-correlation is written as exactly zero.
 *   Samples      complex, [n_channels][n_inputs][row_stride] with re, im
 *                interleaved; CORR_CI8 = int8 re, int8 im (2 B per sample),
 *                CORR_CF32 = float re, float im (8 B per sample), CORR_CI4 =
 *                one byte, re in the high nibble (1 B per sample).
 *   Memory       The caller owns every device buffer, including the workspace
 *                (size from corr_workspace_bytes); libcorr never allocates
 *                device memory.  The library owns only the host-side plan.
 *                All device work is queued on the stream given at creation;
 *                inputs must stay valid until the stream passes the call.
 *   Errors       Every call returns a corr_status; out-parameters are written
 *                only on CORR_OK; no C++ exception crosses this interface.
 *                A HIP error (launch failure now, or a device fault found at
 *                the next synchronising call) returns CORR_E_HIP and puts the
 *                plan in an error state: every later call except
 *                corr_destroy returns CORR_E_STATE.
 *   Threading    A plan is used by one host thread at a time.  Different plans
 *                may be used concurrently from different threads and streams.
 */
#ifndef CORR_H
#define CORR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct corr_plan corr_plan;

typedef enum {
    CORR_OK = 0,
    CORR_E_INVAL = -1,        /* bad argument or configuration            */
    CORR_E_WORKSPACE = -2,    /* workspace missing, too small, misaligned */
    CORR_E_HIP = -3,          /* HIP runtime error (plan now in error)    */
    CORR_E_STATE = -4,        /* plan in error state, or wrong call order */
    CORR_E_OVERFLOW = -5,     /* accumulation would exceed the int32/FP32 bound */
    CORR_E_SEQ = -6,          /* sample-block sequence gap or duplicate   */
    CORR_E_BUSY = -7,         /* ring buffer full / result not ready      */
    CORR_E_UNSUPPORTED = -8,  /* valid request this build does not handle */
    CORR_E_CORRUPT = -9,      /* a workspace guard band was overwritten (a
                                 kernel wrote outside its region); the plan
                                 is now in error                          */
    CORR_STATUS_MIN_ = -2147483647 - 1  /* never returned: gives the enum the
                                 whole int32 range, so that any int a caller
                                 passes to corr_status_str is a value of the
                                 type in C++ as in C                        */
} corr_status;

typedef enum {
    CORR_CF32 = 0,            /* complex float32 pairs                   */
    CORR_CI8 = 1,             /* complex int8 pairs                       */
    CORR_CI4 = 2              /* complex 4-bit, one byte per sample: re in
                                 bits 7..4, im in bits 3..0, two's
                                 complement (the "1-byte" mode of Sec. 5);
                                 int8 engine, max_abs <= 7, X-engine input
                                 only (fft_size 0); rows and the base
                                 pointer 16-byte aligned, else
                                 CORR_E_UNSUPPORTED                      */
} corr_sample_t;

typedef enum {
    CORR_X_FP32 = 0,          /* plain FP32 vector FMA, FP32 accumulation  */
    CORR_X_I8 = 1,            /* int8 MFMA, int32 accumulation (CI8 only)  */
    CORR_X_F16 = 2,           /* FP16 MFMA, FP32 accumulation (CF32 input,
                                 staged unscaled, |x| < 65504)             */
    CORR_X_F8 = 3,            /* OCP FP8 E4M3 MFMA, FP32 accumulation (CF32
                                 input staged with a power-of-two per-channel
                                 scale s_c: the largest with s_c * max|x| <=
                                 448, kept in [2^-60, 2^60]; the epilogue
                                 multiplies by 1/s_c^2).  F16 and F8 plans
                                 with more than 65535 inputs or channels
                                 return CORR_E_UNSUPPORTED.                */
    CORR_X_FP32M = 4          /* FP32 on the matrix cores
                                 (v_mfma_f32_16x16x4_f32), FP32 accumulation;
                                 CF32 input only, no F-stage; rows and base
                                 16-byte aligned (else corr_correlate returns
                                 CORR_E_UNSUPPORTED).  Products and sums are
                                 FP32, in the matrix core's order; exact for
                                 integer samples under the FP32 bound.     */
} corr_engine_t;

/* F-stage input formats (corr_config.volt_format). */
typedef enum {
    CORR_VOLT_R8 = 0,         /* real int8 samples, 1 byte; real DFT of
                                 fft_size = 2*n_channels (Sec. 2, Sec. 4)    */
    CORR_VOLT_CW16 = 1,       /* complex, 5-bit re and 5-bit im in two's
                                 complement in a 16-bit word, re = bits 9..5,
                                 im = bits 4..0, bits 15..10 ignored (the
                                 recorded format of Sec. 3; bit positions are
                                 this library's reading); complex DFT of
                                 fft_size = n_channels                       */
    CORR_VOLT_CB8 = 2         /* complex "1-byte" mode (Sec. 5): 4-bit re in
                                 bits 7..4, 4-bit im in bits 3..0, two's
                                 complement; complex DFT of fft_size =
                                 n_channels                                  */
} corr_volt_t;

typedef struct {
    int32_t n_inputs;         /* N_I >= 1                                   */
    int32_t n_channels;       /* N_C >= 1                                   */
    int32_t fft_size;         /* 0: X-engine only.  Else the F-stage's DFT
                                 length: 2*n_channels for real input (this
                                 build implements 256), n_channels for
                                 complex input (this build implements 128);
                                 other lengths return CORR_E_UNSUPPORTED     */
    int32_t sample_type;      /* corr_sample_t of corr_correlate's input     */
    int32_t engine;           /* corr_engine_t                               */
    int32_t max_abs;          /* > 0: samples are integers with |re|,|im| <=
                                 max_abs (sets the overflow and exactness
                                 bounds; F-stage output is clipped to it).
                                 0: float samples (FP32/F16/F8 engines)      */
    float requant_scale;      /* F-stage: q = clip(rne(s * X_k), +-max_abs)  */
    int32_t fp64_longrun;     /* nonzero: keep an FP64 long-run accumulator  */
    int64_t ring_samples;     /* F-stage: ring capacity in time samples per
                                 channel (one sample per FFT block).
                                 F16/F8: > 0 = convert each call in chunks of
                                 at most this many samples into a staging
                                 buffer, then correlate the chunk; 0 = no
                                 staging buffer: the X-engine converts while
                                 it loads (one pass over the CF32 samples;
                                 rows must start 8-byte aligned, else
                                 corr_correlate returns CORR_E_UNSUPPORTED;
                                 F8 scales s_c by the call's samples).  Both
                                 give the same sums when a chunk holds the
                                 whole call.                                 */
    int32_t volt_format;      /* corr_volt_t of corr_channelise's input (0
                                 when fft_size is 0)                         */
    int32_t pfb_taps;         /* real F-stage only: 0 or 1 = plain DFT; P > 1
                                 = polyphase filterbank of P taps (Sec. 6.1
                                 suggests one against the DFT's leakage; this
                                 build implements P = 4, other P return
                                 CORR_E_UNSUPPORTED): block b's transform input
                                 is y_b[n] = sum_{p<P} h[pN+n] x[(b+p)N+n],
                                 h[m] = w[m] sinc((m - (PN-1)/2)/N) with the
                                 Hamming window w[m] = 0.54 - 0.46 cos(2 pi m
                                 / (PN-1)), N = fft_size, m < PN; 0 when
                                 fft_size is 0                               */
} corr_config;

/* Bytes of device workspace a plan needs for `cfg`.  Host only.  The
 * workspace holds the plan's regions, the integration accumulator first (at
 * offset 0, [n_channels][P][2]), each region padded to 256 bytes and followed
 * by a 256-byte guard band; its last 256 bytes hold the guard check's result
 * (race and overrun detection: see corr_dump). */
corr_status corr_workspace_bytes(const corr_config *cfg, size_t *bytes);

/* Validate `cfg`, carve the caller's workspace (device pointer, >= the size
 * from corr_workspace_bytes, 256-byte aligned) and queue its initialisation
 * on `hip_stream` (a hipStream_t; NULL = default stream).  The plan keeps
 * pointers into the workspace, which must outlive it.  No kernel runs on
 * data yet.  On success *out holds a new plan (owned by the library, freed
 * by corr_destroy). */
corr_status corr_create(const corr_config *cfg, void *d_workspace, size_t ws_bytes,
                        void *hip_stream, corr_plan **out);

/* Free the host plan.  Does not synchronise or touch device memory.  Safe on
 * NULL and on a plan in error state. */
corr_status corr_destroy(corr_plan *plan);

/* F-stage (Sec. 4, steps 1 and 2; the unpack transpose is fused into it).
 * d_volt: device samples in cfg.volt_format, [n_blocks*fft_size][n_inputs],
 * time-major with the input index fastest (the aggregated order of Sec. 3):
 * int8 bytes (CORR_VOLT_R8), 16-bit words (CORR_VOLT_CW16) or bytes
 * (CORR_VOLT_CB8).  Each block of fft_size samples of each input is
 * transformed by a DFT (forward sign, unnormalised, no window).  Real input:
 * channels k = 0..fft_size/2-1 are kept (DC kept, Nyquist dropped).  Complex
 * input (Sec. 2: N_C samples give N_C channels): every k = 0..fft_size-1, in
 * natural order (DC first, negative frequencies in the upper half).  With
 * cfg.pfb_taps = P > 1, d_volt holds n_blocks + P - 1 blocks (the caller
 * repeats the last P - 1 blocks of one call at the start of the next) and
 * spectrum b is that of y_b (see corr_config.pfb_taps); n_blocks counts the
 * spectra.  The spectra are scaled by requant_scale, rounded half to even,
 * clipped to +-max_abs and appended as one CI8 time sample per block to the
 * ring [n_channels][n_inputs][.] in the workspace.
 * first_seq: sequence number of the first block; it must equal the number
 * that follows the previous call's last block (any value on the first call
 * or after corr_seq_reset), else CORR_E_SEQ and nothing is done.
 * CORR_E_BUSY if the ring lacks room for n_blocks more samples (correlate
 * first).  d_spectra_dbg: optional device float32 [n_channels][n_inputs]
 * [n_blocks][2] that receives the spectra before requantisation (NULL in
 * production; parity tests use it).  Asynchronous. */
corr_status corr_channelise(corr_plan *plan, const void *d_volt, int64_t n_blocks,
                            uint64_t first_seq, float *d_spectra_dbg);

/* Aggregation of capture streams (Sec. 3).  d_records: device uint16
 * [n_streams][n_records][1 + words_per_record]: in every stream, each record
 * is one marker/counter word followed by one sample word per receiver input.
 * The marker words are dropped and the streams interleaved so that the
 * n_streams*words_per_record samples of one time instant are adjacent:
 * d_out[r][s*words_per_record + w] = record r of stream s, word 1 + w
 * (device uint16 [n_records][n_streams*words_per_record], caller-owned; the
 * corr_channelise input for CORR_VOLT_CW16).  The marker is read as a 16-bit
 * record counter: d_bad_records (optional device uint32, may be NULL) is
 * incremented once per record whose counter is not (first_counter + r) mod
 * 2^16 in at least one stream; the data are copied regardless.  No plan
 * needed; asynchronous on hip_stream (NULL = default stream).  Any shape is
 * accepted; the prototype's shape is fastest (words_per_record = 16,
 * n_streams <= 4, n_records a multiple of 8, d_records and d_out 16-byte
 * aligned).
 * CORR_E_INVAL for n_streams or words_per_record < 1, n_records < 0, or a
 * NULL buffer with n_records > 0; CORR_E_HIP if the launch fails. */
corr_status corr_aggregate_w16(const uint16_t *d_records, int32_t n_streams, int32_t words_per_record,
                               int64_t n_records, uint32_t first_counter, uint16_t *d_out,
                               uint32_t *d_bad_records, void *hip_stream);

/* The paper's three CMAC designs (Sec. 4, Tables 2-4), kept as described so
 * that their comparison can be repeated on this hardware beside the tiled
 * engines of corr_correlate.  d_spectra: device complex float32
 * [n_samples][n_inputs][n_channels][2] (channel fastest: the FFT output order
 * of Fig. 1, one thread per channel).  Adds (accumulate != 0) or writes, for
 * every channel c and pair j <= i, sum over the n_samples of x_i conj(x_j)
 * (FP32 FMA, sequential in time) into d_out [n_channels][P][2] float32 (P =
 * n_inputs(n_inputs+1)/2, b(i,j) = i(i+1)/2 + j; autos get im = 0).
 *   design CORR_DESIGN_PP (group 1): pair parallel, 2 global reads per
 *     product, pair decoded from a constant-memory table;
 *   CORR_DESIGN_GP (group 2 or 4): group parallel, 2G reads per G^2
 *     products, i-axis values shared through LDS with a barrier per sample;
 *   CORR_DESIGN_HG (group 2 or 4): hybrid group, G+1 reads per G products,
 *     LDS used as register space (no barrier), redundant half exits.
 * CORR_E_INVAL for an unknown design, a group not allowed for it, n_inputs not
 * a multiple of the group, n_inputs or n_channels < 1, n_samples < 0 or a
 * NULL buffer; CORR_E_UNSUPPORTED for n_inputs > 128; CORR_E_HIP if the
 * table upload or the launch fails.  No plan needed;
 * asynchronous on hip_stream (NULL = default stream), except that the first
 * call on a device uploads the 33 KB pair table to constant memory
 * synchronously (so it must not be the first call inside a stream capture). */
typedef enum {
    CORR_DESIGN_PP = 0,
    CORR_DESIGN_GP = 1,
    CORR_DESIGN_HG = 2
} corr_design_t;
corr_status corr_cmac_design(int32_t design, int32_t group, const float *d_spectra, int64_t n_samples,
                             int32_t n_inputs, int32_t n_channels, float *d_out, int32_t accumulate,
                             void *hip_stream);

/* Accept any first_seq on the next corr_channelise call. */
corr_status corr_seq_reset(corr_plan *plan);

/* Checkpoint and resume of a long run (Fig. 1: visibilities dumped after
 * each interval and kept; Sec. 5: continuous operation).  What a plan needs
 * to continue is its FP64 long-run sum (corr_dump with CORR_DUMP_LONGRUN),
 * the number of samples folded into it and the F-stage's next block
 * sequence number; the integration accumulator and the ring are not kept.
 * corr_state writes those two numbers (*seq_valid 0: no block seen since
 * creation or corr_seq_reset).  Host only; any out pointer may be NULL. */
corr_status corr_state(const corr_plan *plan, int64_t *n_long, uint64_t *next_seq, int32_t *seq_valid);

/* Load a checkpoint into a plan with the same configuration (and
 * fp64_longrun set): the long-run sum from `longrun` ([n_channels][P][2]
 * float64, host memory if src_is_device == 0, else device), the sample count
 * n_long (>= 0) and the sequence state.  The integration accumulator and the
 * ring are emptied.  Synchronises the plan's stream.  CORR_E_INVAL for a plan
 * without a long-run sum or a NULL source; CORR_E_STATE for a plan in error. */
corr_status corr_restore(corr_plan *plan, const void *longrun, int32_t src_is_device, int64_t n_long,
                         uint64_t next_seq, int32_t seq_valid);

/* X-engine (Sec. 4 "third step"): for every channel and every pair j <= i,
 * add sum over the n_samples time samples of x_i conj(x_j) to the plan's
 * integration accumulator.
 * d_samples: device samples of cfg.sample_type, [n_channels][n_inputs]
 * [row_stride] (row_stride in samples; 0 means n_samples), of which the first
 * n_samples of each row are used.  d_samples == NULL correlates the samples
 * the F-stage has put in the ring (n_samples and row_stride are then
 * ignored) and empties the ring; on a plan without an F-stage, NULL is
 * accepted only with n_samples == 0 (an empty pass, nothing is done).
 * CORR_E_OVERFLOW (before any launch) if, for integer samples, the samples
 * accumulated since the last reset would exceed 2*max_abs^2*n <= 2^31-1 with
 * the int32 engine (2^31-1 over 256 for CORR_CI4, whose sums run at 256
 * times V inside the engine), or 2^24 with the FP32 engine on integer data
 * (exact FP32 sums).  Asynchronous. */
corr_status corr_correlate(corr_plan *plan, const void *d_samples, int64_t n_samples,
                           int64_t row_stride);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * X-engine pass of corr_correlate without a plan or workspace.  cfg: an
 * X-only configuration (fft_size 0, no long-run accumulator) of the int8
 * (CORR_X_I8) or plain FP32 engine; CORR_E_UNSUPPORTED for the FP16/FP8
 * engines.  d_samples: as for corr_correlate ([n_channels][n_inputs]
 * [row_stride], row_stride 0 = n_samples).  d_out: the caller's device
 * accumulator [n_channels][P][2] (int32 for CORR_X_I8, float32 for
 * CORR_X_FP32): the pass is stored into it (accumulate == 0) or added to it
 * (accumulate != 0; the caller then keeps the total sample count within the
 * overflow bound, which is checked here for n_samples only).  The same
 * kernels as corr_correlate give bit-identical results.  Its K-split partial
 * tiles (written by the pass, then added in split order into d_out by a
 * reduction kernel) live in a fixed device array of
 * CORR_STATIC_SCRATCH_BYTES (64 MiB) inside the library, one per GPU, held
 * until the process ends; its address is looked up on the first call on each
 * device, which must be the current device and the stream's.  No device
 * memory is allocated or freed, and nothing in the array needs clearing
 * between calls.  CORR_E_WORKSPACE if the request needs more than that
 * array (K-split partials of split * n_channels * P * 8 bytes, for small
 * arrays with few channels); CORR_E_INVAL / CORR_E_OVERFLOW /
 * CORR_E_UNSUPPORTED as for corr_correlate; CORR_E_HIP if the address lookup
 * or a launch fails.
 * Asynchronous on hip_stream (NULL = default stream).  Every call on a GPU
 * shares that GPU's array: calls that overlap in time on one GPU (other
 * streams, other threads) race and must be serialised by the caller. */
#define CORR_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
corr_status corr_correlate_static(const corr_config *cfg, const void *d_samples, int64_t n_samples,
                                  int64_t row_stride, void *d_out, int32_t accumulate, void *hip_stream);

/* corr_dump `what` flags. */
#define CORR_DUMP_INTEG    1  /* copy the integration accumulator to dst      */
#define CORR_DUMP_LONGRUN  2  /* copy the FP64 long-run accumulator to dst    */
#define CORR_DUMP_FOLD     4  /* first add the integration into the long-run  */
#define CORR_DUMP_NO_RESET 8  /* keep the integration accumulator             */

/* Read the accumulators (Fig. 1): optionally fold the integration accumulator
 * into the FP64 long-run sum (L += V, exact for integer V while |L| < 2^53),
 * copy the integration (INTEG) or long-run (LONGRUN, exclusive with INTEG)
 * triangle to dst ([n_channels][P][2] of the accumulator's type; host memory
 * if dst_is_device == 0, else device), then reset the integration
 * accumulator and its sample count unless NO_RESET.  Raw sums are returned;
 * dividing by *n_samples_out is the caller's choice.  Synchronises the
 * plan's stream, so device faults surface here as CORR_E_HIP -- except for a
 * plain reset (no INTEG, LONGRUN or FOLD flag), which queues nothing and
 * returns at once.  A dump that waits also checks the workspace's guard
 * bands (filled with a fixed pattern before the plan's first kernel): a band
 * that changed means some kernel wrote outside its region, and the dump
 * returns CORR_E_CORRUPT (the copy has been made; the plan is in error).
 * *n_samples_out: time samples accumulated in the integration (before reset).
 * *exact_out: 1 if every sum copied to dst is provably exact, else 0: for
 * INTEG, integer samples on the int8 or FP32 engine (within the bounds
 * above); for LONGRUN, the same and 2 max_abs^2 n <= 2^53 over the n samples
 * folded so far.  Either out pointer may be NULL. */
corr_status corr_dump(corr_plan *plan, int32_t what, void *dst, int32_t dst_is_device,
                      int64_t *n_samples_out, int32_t *exact_out);

/* Copy the F-stage samples waiting in the ring (not yet correlated) to dst
 * as dense CI8 [n_channels][n_inputs][n][2], n = *n_samples_out, host memory
 * if dst_is_device == 0, else device; dst must hold n_channels * n_inputs *
 * ring_samples * 2 bytes.  For inspection and parity tests of the F-stage
 * output.  Synchronises the plan's stream. */
corr_status corr_ring_read(corr_plan *plan, void *dst, int32_t dst_is_device, int64_t *n_samples_out);

/* FP16 / FP8 engines: copy the last chunk staged by corr_correlate to host
 * dst as dense [n_channels][n_inputs][n][2] elements (binary16, or E4M3
 * bytes), n = *n_samples_out, and, if scales != NULL, the per-channel FP8
 * scales s_c (1 for FP16) to host scales[n_channels].  dst must hold
 * n_channels * n_inputs * ring_samples * 2 elements.  For parity tests of the
 * conversion.  Synchronises the plan's stream.  CORR_E_STATE for a plan
 * with ring_samples == 0 (nothing is staged). */
corr_status corr_stage_read(corr_plan *plan, void *dst, float *scales, int64_t *n_samples_out);

/* Bytes of one integration dump (what = CORR_DUMP_INTEG) or long-run dump. */
corr_status corr_dump_bytes(const corr_plan *plan, int32_t what, size_t *bytes);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of integration jobs.
 *
 * Jobs from streams with different input and channel counts arrive at any
 * time (the real-time operation of Sec. 5; the batching of many cycles per
 * GPU call, Sec. 5).  corr_sched_submit never blocks: a job waits in a FIFO
 * queue until its HBM footprint fits in the caller's arena (its samples when
 * a fill callback produces them, its result when the destination is host
 * memory) and one of 64 queue slots is free.  An admitted job is published
 * on a job queue in the arena's head; a persistent int8 X-engine grid (as
 * many workgroups as the GPU holds at once) takes work items -- (channel,
 * 128-row baseline tile) pairs -- round robin from every published job
 * with unclaimed items, so jobs that arrive while others run are taken up by
 * the grid already on the device, and their work overlaps.  No per-job plan is created and no kernel
 * is launched per job: the grid closes as a whole once the queue has been
 * idle for 0.1 ms, and a new one is launched when work is published after
 * that.  A running grid leaves 16 workgroup slots free; other work on the
 * GPU (the runtime's copies, the per-job path below, fill callbacks) runs
 * there.  The job's device result is complete when its last
 * item is done (the grid then writes a completion word in pinned host memory
 * that the scheduler polls); a host destination then receives a copy, and
 * the job is complete when that copy has landed (the latency end point).
 * Samples whose rows are not 16-byte aligned (caller buffers with an odd row
 * stride) are correlated through a per-job plan on one of n_streams streams
 * instead.  A job whose footprint exceeds the whole arena is refused at
 * submission (CORR_E_WORKSPACE).  The scheduler allocates, besides its host
 * objects, 264 KB of pinned host memory (completion words and the staging of
 * queue updates); no device memory.
 * ------------------------------------------------------------------------ */
typedef struct corr_sched corr_sched;

/* Writes the job's samples, complex int8 [n_channels][n_inputs][row_stride]
 * (the first n_samples of each row; row_stride >= n_samples is chosen by the
 * scheduler), to device memory d_samples by queueing work on hip_stream;
 * called from the scheduler's thread when the job is admitted; must not
 * block. */
typedef void (*corr_fill_fn)(void *user, uint64_t job_id, void *d_samples, int64_t n_channels,
                             int64_t n_inputs, int64_t n_samples, int64_t row_stride, void *hip_stream);

typedef struct {
    int32_t n_inputs;         /* N_I >= 1                                     */
    int32_t n_channels;       /* N_C >= 1                                     */
    int64_t n_samples;        /* time samples per channel, >= 1               */
    int32_t max_abs;          /* declared bound on |re|, |im| (1..127)        */
    int32_t reserved;
    corr_fill_fn fill;        /* produces the samples on the device, or NULL  */
    void *fill_user;          /* passed to fill                                */
    const void *d_samples;    /* used when fill == NULL: caller's device
                                 samples [n_channels][n_inputs][row_stride]
                                 (e.g. a stream's ring buffer), valid until
                                 the job completes                            */
    int64_t row_stride;       /* samples between rows of d_samples; 0 means
                                 n_samples (ignored with fill)                */
    void *dst;                /* int32 [n_channels][P][2] result, valid until
                                 the job completes                            */
    int32_t dst_is_device;    /* 1: dst is device memory; 0: host memory
                                 (pinned, else the copy blocks the scheduler) */
    int32_t reserved2;
} corr_job_desc;

/* Seconds on the clock the scheduler stamps completions with (monotonic). */
double corr_sched_now(void);

/* d_arena: caller-owned device memory (256-byte aligned) holding the job
 * queue (its first 35 KB) and the job footprints; n_streams: streams for
 * jobs on the per-job path (1..16).  All streams are of default priority,
 * created and owned by the scheduler.  CORR_E_WORKSPACE if the arena is
 * NULL, misaligned or smaller than the queue. */
corr_status corr_sched_create(void *d_arena, size_t arena_bytes, int32_t n_streams, corr_sched **out);

/* Queue a job.  t_arrival: its arrival time on corr_sched_now()'s clock (the
 * latency origin).  *job_id receives its id.  Never blocks. */
corr_status corr_sched_submit(corr_sched *s, const corr_job_desc *job, double t_arrival, uint64_t *job_id);

/* CORR_E_BUSY while job_id is queued or running.  Once it is complete:
 * CORR_OK (or the job's own error status), *n_samples_out, *t_admit (its
 * admission), *t_device (its integration complete in device memory, seen by
 * the scheduler) and *t_done (its completion: the result in the job's
 * destination) are written and the job record is released; a second poll of
 * the same id gives CORR_E_INVAL.  Any out pointer may be NULL. */
corr_status corr_sched_poll(corr_sched *s, uint64_t job_id, int64_t *n_samples_out, double *t_admit,
                            double *t_device, double *t_done);

/* stats[0..7] = submitted, admitted, completed, failed, queued now, running
 * now, peak arena bytes in use, arena bytes. */
corr_status corr_sched_stats(corr_sched *s, int64_t stats[8]);

/* Wait for every queued and running job, then free the scheduler. */
corr_status corr_sched_destroy(corr_sched *s);

/* Static description of a status code. */
const char *corr_status_str(corr_status s);

#ifdef __cplusplus
}
#endif

#endif /* CORR_H */
