/*
 * ppf.h - C ABI of the MI355X polyphase filter bank (PPF) library, libppf.so.
 *
 * The PPF (Adamek, Novotny, Armour, "The Implementation of a Real-Time
 * Polyphase Filter", section 2) is a FIR filter applied per channel across
 * N channels (Eq. 1, with T taps), followed by an N-point DFT of every
 * filtered block (section 3: the FIR is followed by a library FFT).
 * For an input x of (M+T-1)*N complex samples and real prototype
 * coefficients h of T*N values, spectrum m (0 <= m < M) is
 *
 *     u[m][c] = sum_{t=0}^{T-1} h[t*N + c] * x[(m+t)*N + c]
 *     X[m][k] = sum_{c=0}^{N-1} u[m][c] * exp(-2*pi*i*c*k/N)
 *
 * i.e. segment t of the prototype weights input block m+t (per channel,
 * Eq. 1 with b_i = h[(T-1-i)*N + c]). The transform is the unnormalised
 * forward DFT with bins in natural order. Only valid spectra are produced:
 * M spectra need (M+T-1)*N input samples.
 *
 * Conventions for every entry point:
 *  - Plain C: no exceptions cross the ABI; sizes are 64-bit where they can
 *    exceed 2^31.
 *  - Status: functions returning int return PPF_OK (0) or a negative
 *    ppf_status. Functions returning a handle return NULL on error.
 *    Either way the code of the most recent failure on the calling host
 *    thread is kept for ppf_last_error() and a message for
 *    ppf_last_error_message().
 *  - Arguments are validated before any HIP call is made; an invalid
 *    argument never launches work.
 *  - "Device pointer" means memory of the current HIP device (hipMalloc,
 *    torch CUDA tensors). The caller owns it and keeps it valid until the
 *    work that uses it has completed on the plan's stream.
 *  - Complex data is interleaved (re, im) in time order, so channel c of
 *    block b is sample b*N + c (channels contiguous).
 *  - Supported sizes on the GPU: N a power of two in [16, 16384] and
 *    1 <= T <= 64. Other sizes return PPF_ERR_UNSUPPORTED.
 */
#ifndef PPF_H
#define PPF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum ppf_status {
    PPF_OK = 0,
    PPF_ERR_INVALID = -1,     /* NULL handle/pointer, negative count, overlap, bad enum */
    PPF_ERR_UNSUPPORTED = -2, /* N or T outside the supported set, or a mode not built */
    PPF_ERR_ALIGN = -3,       /* a data pointer is not 16-byte aligned */
    PPF_ERR_NOMEM = -4,       /* device or host allocation failed */
    PPF_ERR_BUDGET = -5,      /* an admission would exceed the state budget */
    PPF_ERR_HIP = -6,         /* a HIP runtime call or kernel launch failed */
    PPF_ERR_BUSY = -7         /* the object still has work in flight */
};

/* Element types. Complex types are interleaved (re, im) pairs. */
enum ppf_dtype {
    PPF_C32 = 0, /* complex float32, 8 bytes per sample */
    PPF_C16 = 1, /* complex float16, 4 bytes per sample */
    PPF_CI8 = 2, /* complex int8, 2 bytes per sample */
    PPF_R32 = 3, /* real float32 (coefficients) */
    PPF_R16 = 4  /* real float16 (coefficients) */
};

/* How the DFT stages are computed. */
enum ppf_fft_mode {
    PPF_FFT_F32 = 0,      /* FP32 radix stages on the vector ALUs */
    PPF_FFT_MFMA_F16 = 1  /* radix-16 stages as FP16 MFMA, FP32 accumulate */
};

/* Windows of the prototype-filter designer (ppf_design_coeffs). */
enum ppf_window {
    PPF_WIN_RECT = 0,     /* 1 */
    PPF_WIN_HAMMING = 1,  /* 0.54 - 0.46 cos(2 pi j/(L-1)) */
    PPF_WIN_HANN = 2,     /* 0.5 - 0.5 cos(2 pi j/(L-1)) */
    PPF_WIN_KAISER = 3,   /* I0(beta sqrt(1 - r^2)) / I0(beta), r = 2j/(L-1) - 1 */
    PPF_WIN_USER = 4      /* L values given by the caller */
};

/* Execution paths a plan can use (ppf_plan_set_path / ppf_plan_query). */
enum ppf_path {
    PPF_PATH_AUTO = 0,     /* library's choice */
    PPF_PATH_FUSED = 1,    /* one kernel: FIR presum and FFT on chip */
    PPF_PATH_TWO_PASS = 2  /* FIR kernel then FFT kernel through a workspace */
};

/* Keys for ppf_plan_query. */
enum ppf_query {
    PPF_Q_N = 0,               /* channels */
    PPF_Q_TAPS = 1,            /* taps T */
    PPF_Q_PATH = 2,            /* ppf_path in use (never AUTO) */
    PPF_Q_WORKSPACE_BYTES = 3, /* device workspace owned by the plan */
    PPF_Q_IN_TYPE = 4,         /* ppf_dtype of the input */
    PPF_Q_FFT_MODE = 5,        /* ppf_fft_mode */
    PPF_Q_COEFF_SHIFT = 6,     /* s: stored coefficients are h * 2^s */
    PPF_Q_FUSED_AVAILABLE = 7  /* 1 if the fused path exists for this N, T */
};

typedef struct ppf_plan_s* ppf_plan_t;

/*
 * ppf_plan - create an immutable FP32 plan for N channels and T taps.
 *
 * coeffs: host pointer to T*N float32 prototype coefficients, h[t*N + c]
 *         weighting channel c of block m+t (the constant response function
 *         of section 2). Copied; the caller keeps ownership.
 * The plan uploads the coefficients and computes the DFT twiddles
 * exp(-2*pi*i*k/N) in FP64 on the GPU, rounded once to FP32. Input is
 * complex FP32, output complex FP32, FFT in FP32.
 * Returns NULL on error (PPF_ERR_INVALID for NULL coeffs,
 * PPF_ERR_UNSUPPORTED for N or T outside the supported set, PPF_ERR_HIP or
 * PPF_ERR_NOMEM for device failures).
 */
ppf_plan_t ppf_plan(int n_channels, int taps, const float* coeffs);

/*
 * ppf_plan_ex - plan with explicit precision (the reduced-precision form).
 *
 * coeff_type: PPF_R32 (coeffs is float32[T*N]) or PPF_R16 (float16[T*N]).
 * coeff_shift: the stored coefficients are h * 2^coeff_shift; the FP32
 *         accumulation is scaled by 2^-coeff_shift. Must be 0 for PPF_R32;
 *         0..30 for PPF_R16.
 * in_type: PPF_C32, PPF_C16 or PPF_CI8. Inputs are converted exactly to
 *         FP32 in registers as they are loaded (by the fused kernel where
 *         the shape has one, else by the FIR pass of the two-pass form);
 *         the FIR accumulates in FP32. Output is always C32.
 * fft_mode: PPF_FFT_F32 or PPF_FFT_MFMA_F16 (PPF_ERR_UNSUPPORTED where the
 *         MFMA stages are not built for N). The matrix-core mode is built
 *         for N = 4096 = 16^3 (three radix-16 stages), N = 1024 = 4 * 16^2
 *         (a radix-4 stage in FP32, then two radix-16 stages) and N = 256 =
 *         16^2, T <= 16, PPF_R16 coefficients and PPF_CI8 or PPF_C16 input;
 *         the samples enter the FP16 stages scaled by a power of two chosen
 *         so that no stage input can overflow for any input value of that
 *         type (|x| <= 128 for int8, 65504 for FP16). Any other combination
 *         is PPF_ERR_UNSUPPORTED.
 */
ppf_plan_t ppf_plan_ex(int n_channels, int taps, const void* coeffs, int coeff_type,
                       int coeff_shift, int in_type, int fft_mode);

/*
 * ppf_set_stream - HIP stream (a hipStream_t passed as void*) on which the
 * calling host thread enqueues its work on this plan; NULL selects the null
 * stream (the default). The binding belongs to the calling thread, not to
 * the plan: the plan is not modified, and threads that bind different
 * streams may use one plan at the same time.
 */
int ppf_set_stream(ppf_plan_t plan, void* hip_stream);

/*
 * ppf_plan_set_path - force a path before the plan is used (tests and
 * benchmarks). PPF_ERR_UNSUPPORTED if the path does not exist for N, T.
 * The one call that changes a plan: make it before the plan is shared.
 */
int ppf_plan_set_path(ppf_plan_t plan, int path);

/* ppf_plan_query - read a plan property (enum ppf_query) into *value. */
int ppf_plan_query(ppf_plan_t plan, int key, long long* value);

/*
 * ppf_execute - the batch PPF, enqueued asynchronously on the plan's stream.
 *
 * in:  device pointer, (nspectra + T - 1) * N samples of the plan's input type.
 * out: device pointer, nspectra * N complex FP32 spectra, out[m*N + k] = X[m][k].
 * Both 16-byte aligned (else PPF_ERR_ALIGN) and non-overlapping (else
 * PPF_ERR_INVALID). nspectra == 0 is a successful no-op; nspectra < 0 is
 * PPF_ERR_INVALID. The work goes to the calling thread's stream for the
 * plan (ppf_set_stream). Calls from several threads on one plan are safe:
 * the two-pass path keeps one device workspace (128 MiB; 512 MiB for
 * N >= 8192) per HIP stream, allocated on that stream's first two-pass
 * call and freed with the plan.
 */
int ppf_execute(ppf_plan_t plan, const void* in, void* out, long long nspectra);

/*
 * ppf_execute_host - the batch PPF on host-resident data (the single mode
 * of section 3, whose throughput includes the PCIe transfers: the M_b
 * measure of Table 2), enqueued asynchronously on the plan's stream.
 *
 * host_in:  host pointer, (nspectra + T - 1) * N samples of the plan's
 *           input type.
 * host_out: host pointer, nspectra * N complex FP32 spectra.
 * chunk_spectra: spectra per pipeline chunk (0 selects about 192 MiB of
 *           input per chunk).
 *
 * The batch is cut into chunks of consecutive spectra; chunk i's input
 * (its spectra plus the T-1 blocks that follow) is copied to a device
 * staging buffer on a copy stream while earlier chunks are transformed on
 * the plan's stream and copied back on another copy stream. The plan owns
 * three pairs of staging buffers (allocated on first use, grown to the
 * chunk size), so up to three chunks are in flight. The plan's stream
 * completes when every spectrum is in host_out. Host buffers must stay
 * valid until then and should be page-locked (hipHostMalloc) for the
 * copies to run asynchronously at full rate.
 * Errors as ppf_execute, plus PPF_ERR_NOMEM for the staging buffers.
 * The staging buffers belong to the plan: one ppf_execute_host at a time
 * per plan (other entry points may run beside it).
 */
int ppf_execute_host(ppf_plan_t plan, const void* host_in, void* host_out, long long nspectra,
                     long long chunk_spectra);

/*
 * ppf_execute_power - detection after the filter bank: the power of every
 * bin summed over K consecutive spectra (the screening step the filter bank
 * feeds, section 1), computed in the transform's epilogue so the complex
 * spectra never reach memory. Enqueued asynchronously on the plan's stream.
 *
 * in:        device pointer, (nspectra + T - 1) * N samples of the input type.
 * out_power: device pointer, (nspectra / K) * N floats,
 *            out_power[j*N + k] = sum_{i<K} |X[j*K + i][k]|^2.
 * K >= 1 and nspectra a multiple of K (else PPF_ERR_INVALID). K above 2^28,
 * or K*N above 2^24 on the two-pass path (whole groups of K spectra pass
 * through its workspace), is PPF_ERR_UNSUPPORTED. Alignment, overlap and
 * nspectra rules as ppf_execute. Plans in the matrix-core mode detect in
 * the same epilogue, from their FP32-accumulated spectra; FP32-DFT plans
 * with FP16 or int8 input detect in the two-pass form.
 */
int ppf_execute_power(ppf_plan_t plan, const void* in, float* out_power, long long nspectra, int K);

/*
 * ppf_execute_noalloc - ppf_execute that allocates nothing, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, hosts that forbid it).
 *
 * Same arguments, stream, layout and errors as ppf_execute. The two-pass
 * path presums into a static device workspace of PPF_NOALLOC_SCRATCH_BYTES
 * (32 MiB, one per GPU, held until the process ends) instead of the
 * per-stream workspace ppf_execute allocates: a two-pass batch whose
 * presums (nspectra * N * 8 bytes) exceed it is PPF_ERR_UNSUPPORTED, with
 * nothing launched (split the batch). Fused and matrix-core plans use no
 * workspace and take any nspectra. Every call on a GPU shares that GPU's
 * workspace: two-pass calls that overlap on one GPU (different streams or
 * threads) race and must be ordered by the caller.
 */
#define PPF_NOALLOC_SCRATCH_BYTES (32u << 20)
int ppf_execute_noalloc(ppf_plan_t plan, const void* in, void* out, long long nspectra);

/* ppf_destroy - wait for every HIP stream the plan has run on, then free the
 * plan. No other call may use the plan meanwhile. NULL is a no-op. */
int ppf_destroy(ppf_plan_t plan);

/*
 * ppf_design_coeffs - prototype coefficients for ppf_plan from the constant
 * response function of section 2: the ideal pass band of one channel is a
 * sinc in time, sampled over L = taps * n_channels points and tapered by a
 * window (the paper uses the Kaiser window, with its parameter unstated):
 *
 *     v[j] = w[j] * sinc((j - (L-1)/2) / n_channels),  sinc(u) = sin(pi u)/(pi u)
 *     coeffs[j] = v[j] / sum_i v[i]                    (gain 1 at DC)
 *
 * so the pass band reaches half amplitude half a bin from the channel
 * centre. w is the window (enum ppf_window) over j = 0 .. L-1; L = 1 gives
 * w = 1. Computed on the current HIP device in FP64 and rounded once to
 * FP32; synchronous (plan time: it allocates and frees device memory).
 *
 * beta:        Kaiser parameter, 0 <= beta <= 60 (PPF_WIN_KAISER only;
 *              ppf_kaiser_beta gives it from a stop-band attenuation).
 * user_window: host pointer, L doubles (PPF_WIN_USER only, else ignored).
 * coeffs:      host pointer, L floats; the caller owns it.
 * n_channels >= 1 and taps >= 1 (any values, not only the sizes a plan
 * supports), else PPF_ERR_INVALID; L above 2^20 is PPF_ERR_UNSUPPORTED.
 * A bad window, beta out of range or not a number, a NULL coeffs, or a
 * NULL user_window for PPF_WIN_USER is PPF_ERR_INVALID, as is a window
 * whose windowed sinc sums to zero or to a value that is not finite.
 */
int ppf_design_coeffs(int n_channels, int taps, int window, double beta, const double* user_window,
                      float* coeffs);

/*
 * ppf_kaiser_beta - Kaiser's empirical rule for the window parameter from
 * the wanted stop-band attenuation A in dB: 0.1102 (A - 8.7) for A > 50,
 * 0.5842 (A - 21)^0.4 + 0.07886 (A - 21) for 21 <= A <= 50, else 0.
 * Host arithmetic only. A not a number or a NULL beta is PPF_ERR_INVALID.
 */
int ppf_kaiser_beta(double atten_db, double* beta);

/* ------------------------------------------------------------------------
 * Stream form.
 *
 * A stream feeds an unbounded sample sequence through a plan in chunks. Its
 * state is the last (T-1)*N input samples (the T-1 past samples of Eq. 1 per
 * channel), kept in device memory. The outputs of successive pushes are
 * exactly the batch PPF over zeros((T-1)*N) ++ chunk_1 ++ chunk_2 ++ ...:
 * a chunk of S*N samples yields S spectra, whatever the chunking (the FIR
 * depends on raw input only, section 2).
 * ---------------------------------------------------------------------- */

typedef struct ppf_stream_s* ppf_stream_t;

/* One chunk: in = nspectra*N samples of the plan's input type (device),
 * out = nspectra*N complex FP32 bins (device), 16-byte aligned, not
 * overlapping. tag is the caller's identifier (used by the server). */
typedef struct ppf_chunk {
    const void* in;
    void* out;
    long long nspectra;
    unsigned long long tag;
} ppf_chunk;

/* ppf_stream_create - new stream on `plan` with a zero history. The plan must
 * outlive the stream. Allocates 2*(T-1)*N samples of device memory.
 * Returns NULL on error. (Streams served by a server come from
 * ppf_server_open_stream instead.) */
ppf_stream_t ppf_stream_create(ppf_plan_t plan);

/* ppf_stream_push - process one chunk, asynchronously. A stream from
 * ppf_stream_create enqueues it on the calling thread's HIP stream for the
 * plan (ppf_set_stream); a server stream queues it at its server (as
 * ppf_server_submit with arrival time "now"). Pushes to one stream are
 * processed in order; push to one stream from one thread at a time.
 * nspectra == 0 is a no-op. */
int ppf_stream_push(ppf_stream_t stream, const ppf_chunk* chunk);

/* ppf_stream_get_history / ppf_stream_set_history - copy the (T-1)*N-sample
 * history to / from host memory (synchronous: waits for the stream's latest
 * push). Saving and restoring it resumes a stream exactly
 * (checkpoint/restore). Server streams: PPF_ERR_UNSUPPORTED. */
int ppf_stream_get_history(ppf_stream_t stream, void* host_dst);
int ppf_stream_set_history(ppf_stream_t stream, const void* host_src);

/* Spectra pushed so far. */
long long ppf_stream_position(ppf_stream_t stream);

/* ppf_stream_destroy - wait for the stream's chunks, free its history and the
 * handle. For a server stream: close it, wait until its chunks are done
 * (PPF_ERR_BUSY or PPF_ERR_HIP, after freeing the handle, if the server
 * failed or stopped first), release its state. NULL is a no-op. */
int ppf_stream_destroy(ppf_stream_t stream);

/* ------------------------------------------------------------------------
 * Serving form.
 *
 * A server runs many streams of possibly different N and T on one GPU with
 * continuous batching: chunks submitted from any host thread are grouped by
 * a scheduler thread into batches as in-flight slots free up, the batch's
 * work for all streams runs as one captured HIP graph (one concurrent
 * branch per plan), and each stream's (T-1)*N-sample history stays in
 * device memory between its chunks. Per stream the outputs equal those of
 * the stream form (and of the batch PPF over the zero-prefixed
 * concatenation of its chunks). Streams are admitted while their state fits
 * the server's device-memory budget.
 * ---------------------------------------------------------------------- */

typedef struct ppf_server_s* ppf_server_t;

typedef struct ppf_server_stats_s {
    long long chunks_done;        /* chunks completed since the last reset */
    long long spectra_done;
    long long bytes_in_done;      /* input bytes of completed chunks */
    long long batches;            /* batches launched */
    long long admitted;           /* streams admitted (ever) */
    long long rejected;           /* open requests refused for budget */
    long long queued_admissions;  /* open requests that had to wait for budget */
    long long state_bytes_used;   /* budget in use: admitted streams + server buffers */
    long long tags_dropped;       /* completed tags dropped unpolled (beyond 2^22 kept) */
    double p50_us, p99_us, max_us, mean_us;  /* chunk latency: completion seen on the
                                               host minus arrival time (percentiles
                                               from a histogram of 0.4% bins) */
    double elapsed_s;             /* first arrival to last completion */
    double input_gbps;            /* bytes_in_done / elapsed_s / 1e9 */
    double mean_batch_chunks;
    double mean_batch_gpu_us;     /* device time of a batch graph (timing events) */
    double mean_form_us;          /* host time to form a batch */
    double mean_launch_us;        /* host time of the descriptor upload and graph launch */
} ppf_server_stats_t;

/* Host steady clock in nanoseconds (the time base of arrival times). */
long long ppf_clock_ns(void);

/* ppf_server_create - server with a device-memory budget in bytes for its own
 * buffers plus stream state, and 1..4 batches in flight. Starts the
 * scheduler thread. PPF_ERR_BUDGET if the budget cannot hold the server's
 * own buffers: per in-flight batch, a 512 MiB two-pass workspace and its
 * descriptor tables. Returns NULL on error. */
ppf_server_t ppf_server_create(size_t hbm_budget_bytes, int max_inflight);

/* Flags of ppf_server_open_stream_ex. */
enum ppf_open_flags {
    PPF_OPEN_QUEUE = 0,  /* wait in line for budget (ppf_server_open_stream) */
    PPF_OPEN_NOWAIT = 1  /* PPF_ERR_BUDGET instead of waiting */
};

/*
 * ppf_server_open_stream - open a stream of `plan` on the server; *out gets
 * its handle, fed with ppf_stream_push (or ppf_server_submit) and released
 * with ppf_stream_destroy. The plan must be complex FP32 with FP32 DFT
 * stages (else PPF_ERR_UNSUPPORTED), at most 8 distinct plans per server,
 * and plans must outlive the server. The stream's state is two
 * (T-1)*N-sample history buffers plus 4 KiB. If it does not fit the budget
 * now, the stream waits in line and is admitted, in order, when closing
 * streams free budget; chunks pushed meanwhile run once it is admitted.
 * PPF_ERR_BUDGET if the state can never fit (beyond the budget left after
 * the server's own buffers).
 */
int ppf_server_open_stream(ppf_server_t server, ppf_plan_t plan, ppf_stream_t* out);

/* ppf_server_open_stream_ex - as ppf_server_open_stream; with PPF_OPEN_NOWAIT
 * a stream that does not fit now is refused (PPF_ERR_BUDGET). */
int ppf_server_open_stream_ex(ppf_server_t server, ppf_plan_t plan, int flags, ppf_stream_t* out);

/* 1 if the server stream has been admitted, 0 if it is still waiting, <0 on error. */
int ppf_server_stream_admitted(ppf_stream_t stream);

/* ppf_server_submit - ppf_stream_push with an explicit arrival time:
 * arrival_ns on ppf_clock_ns (< 0: now), from which the chunk's latency is
 * measured. Lock-free for the caller (it waits only while 65536 chunks are
 * queued ahead of the scheduler). A chunk of any size up to 2^31 spectra is
 * taken: one larger than a batch can hold (e.g. 16384 spectra at N=4096
 * two-pass) runs as consecutive pieces, and its tag is reported once, when
 * the last piece is done. Device buffers must stay valid until the tag is
 * returned by ppf_server_poll (or ppf_server_drain returns). */
int ppf_server_submit(ppf_stream_t stream, const ppf_chunk* chunk, long long arrival_ns);

/* ppf_server_poll - copy up to max completed chunk tags, in completion
 * order; returns the number copied (>= 0) or an error. The server keeps the
 * latest 2^22 unpolled tags (older ones are counted in tags_dropped). */
int ppf_server_poll(ppf_server_t server, unsigned long long* tags, int max);

/* ppf_server_drain - wait until every submitted chunk has completed;
 * PPF_ERR_BUSY after timeout_s seconds. */
int ppf_server_drain(ppf_server_t server, double timeout_s);

/* ppf_server_close_stream - no further pushes. An admitted stream's pushed
 * chunks still run, and its budget is given back as soon as they are done;
 * a stream closed while waiting for admission leaves the line and its
 * pushed chunks are dropped (their tags are never returned). The handle
 * stays valid until ppf_stream_destroy. */
int ppf_server_close_stream(ppf_stream_t stream);

/* ppf_server_stats - chunk latency p50 and p99 (us) and sustained input
 * GB/s since the last reset; any pointer may be NULL. */
int ppf_server_stats(ppf_server_t server, double* p50_us, double* p99_us, double* gbps);

/* ppf_server_get_stats - every counter above. */
int ppf_server_get_stats(ppf_server_t server, ppf_server_stats_t* out);
int ppf_server_reset_stats(ppf_server_t server);

/* ppf_server_destroy - finish outstanding chunks of admitted streams (chunks
 * of streams still waiting for admission are dropped), stop the scheduler,
 * free everything. Stream handles of the server that are still open then
 * accept only ppf_stream_destroy. NULL is a no-op. */
int ppf_server_destroy(ppf_server_t server);

/* Status of the most recent failure on this host thread (PPF_OK if none). */
int ppf_last_error(void);
/* Human-readable text of the most recent failure on this host thread. */
const char* ppf_last_error_message(void);
/* Static name of a status code. */
const char* ppf_status_str(int status);

#ifdef __cplusplus
}
#endif

#endif /* PPF_H */
