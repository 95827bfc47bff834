/*
 * dks_fft.h -- C ABI of the raw 3-D FFTs on device data.
 *
 * The paper's DKS exposes the FFT it uses for the Poisson solver directly: the
 * user writes data to the device, calls a forward or inverse transform on it
 * and reads the result back (section "DKS", the FFT usage example figure).
 * These entry points give the same operation on the library's Stockham
 * engine: the discrete Fourier transform over a 3-D (or, with extents of 1,
 * 2-D or 1-D) array,
 *
 *   X[k] = sum_j x[j] exp(-+ 2 pi i (jx kx / nx + jy ky / ny + jz kz / nz)),
 *
 * minus sign forward, plus sign inverse, with no normalisation (inverse of
 * forward multiplies by nx ny nz).
 *
 * Conventions (shared with dks_poisson.h: status codes, dtypes, streams):
 *  - Extents: every n_d in [1, 4096] and of the form 2^a 3^b
 *    (DKS_EUNSUPPORTED otherwise); batch >= 1.
 *  - Layout: C-contiguous [batch][nz][ny][nx], x fastest; complex values are
 *    interleaved (re, im) pairs of the dtype.
 *  - Kinds: DKS_FFT_C2C transforms complex arrays both ways, in place
 *    (in == out) or out of place.  DKS_FFT_R2C: forward takes real
 *    [batch][nz][ny][nx] and writes the non-redundant half spectrum
 *    [batch][nz][ny][nx/2 + 1] (complex); inverse takes that half spectrum
 *    and writes the real array (the imaginary parts of the kx = 0 and, for
 *    even nx, kx = nx/2 inputs are ignored).  R2C transforms are out of place
 *    only (in == out is DKS_EINVAL) and leave their input unchanged.
 *  - Memory: every data pointer is device memory owned by the caller; the
 *    plan's workspace (twiddles, plan copies, the inverse R2C's scratch) is
 *    caller-owned too.  All work is enqueued on the caller's stream with no
 *    host synchronisation.
 */
#ifndef DKS_FFT_H
#define DKS_FFT_H

#include "dks_poisson.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { DKS_FFT_C2C = 0, DKS_FFT_R2C = 1 } dks_fft_kind;

typedef struct dks_fft_plan_s* dks_fft_plan_t;

/* Create a plan (host only; touches no device).
 *   nx, ny, nz : extents, x fastest.
 *   batch      : number of consecutive arrays transformed per call.
 *   kind       : DKS_FFT_C2C or DKS_FFT_R2C (forward real-to-complex,
 *                inverse complex-to-real).
 *   dtype      : DKS_F32 or DKS_F64 (real and imaginary parts).
 *   out        : receives the handle, valid until dks_fft_destroy. */
dks_status dks_fft_plan(int nx, int ny, int nz, int batch, dks_fft_kind kind, dks_dtype dtype,
                        dks_fft_plan_t* out);

/* Bytes of device workspace the plan needs (256-byte alignment required). */
dks_status dks_fft_workspace_bytes(dks_fft_plan_t plan, size_t* bytes);

/* Attach the caller-owned workspace (at least dks_fft_workspace_bytes,
 * 256-byte aligned); dks_fft_prepare must follow. */
dks_status dks_fft_set_workspace(dks_fft_plan_t plan, void* workspace, size_t bytes);

/* Write the twiddle tables (computed in FP64, rounded to the dtype) and the
 * device copies of the axis plans into the workspace, on `stream`. */
dks_status dks_fft_prepare(dks_fft_plan_t plan, dks_stream_t stream);

/* Forward transform (exponent sign -), in -> out, on `stream`.  DKS_ESTATE
 * before dks_fft_prepare. */
dks_status dks_fft_forward(dks_fft_plan_t plan, const void* in, void* out, dks_stream_t stream);

/* Inverse transform (exponent sign +, unnormalised), in -> out. */
dks_status dks_fft_inverse(dks_fft_plan_t plan, const void* in, void* out, dks_stream_t stream);

/* Release the plan's host state; the caller's workspace is untouched. */
dks_status dks_fft_destroy(dks_fft_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* DKS_FFT_H */
