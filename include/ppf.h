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
 * in_type: PPF_C32, PPF_C16 or PPF_CI8. Inputs are converted to FP32 in
 *         registers; the FIR accumulates in FP32. Output is always C32.
 * fft_mode: PPF_FFT_F32 or PPF_FFT_MFMA_F16 (PPF_ERR_UNSUPPORTED where the
 *         MFMA stages are not built for N).
 */
ppf_plan_t ppf_plan_ex(int n_channels, int taps, const void* coeffs, int coeff_type,
                       int coeff_shift, int in_type, int fft_mode);

/*
 * ppf_set_stream - HIP stream (a hipStream_t passed as void*) on which the
 * plan's work is enqueued; NULL selects the null stream (the default).
 * Not thread-safe against concurrent ppf_execute on the same plan.
 */
int ppf_set_stream(ppf_plan_t plan, void* hip_stream);

/*
 * ppf_plan_set_path - force a path before the plan is used (tests and
 * benchmarks). PPF_ERR_UNSUPPORTED if the path does not exist for N, T.
 * Not thread-safe; call before the first ppf_execute.
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
 * PPF_ERR_INVALID. Concurrent calls on one plan with different streams
 * are safe only on the fused path (the two-pass path shares the plan's
 * workspace).
 */
int ppf_execute(ppf_plan_t plan, const void* in, void* out, long long nspectra);

/* ppf_destroy - wait for the plan's stream, then free the plan. NULL is a no-op. */
int ppf_destroy(ppf_plan_t plan);

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
