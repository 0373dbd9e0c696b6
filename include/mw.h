/*
 * mw.h -- C ABI of the MI355X (gfx950) McEwen-Wiaux spin spherical-harmonic
 * transform library (libmw.so).
 *
 * The transforms are those of McEwen & Wiaux, "A novel sampling theorem on the
 * sphere" (IEEE TSP 59(12), 2011):
 *   forward  f(theta_t, phi_p) -> sf_lm   (Sec. IV-D, algorithm Forward Transform,
 *                                         Eqs.(flm_wig), (Gmm), (Gmt), (Gmm_convolution))
 *   inverse  sf_lm -> f(theta_t, phi_p)   (Sec. IV-E, algorithm Inverse Transform,
 *                                         Eqs.(f_pfft), (Fmt), (Fmm))
 * on the equiangular grid of Sec. IV-C:
 *   theta_t = pi (2t+1)/(2L-1), t = 0..L-1;   phi_p = 2 pi p/(2L-1), p = 0..2L-2.
 *
 * ---------------------------------------------------------------------------
 * Data layout (all buffers are DEVICE memory owned by the caller)
 *   map    : row-major [t][p], L rows of 2L-1 samples.  The last row (t = L-1)
 *            is the south pole theta = pi, stored as a full ring.  Interleaved
 *            complex128 (re, im) when reality = 0; float64 when reality = 1.
 *   coeffs : complex128 at index l*l + l + m, 0 <= l < L, |m| <= l (L*L entries).
 *            The forward writes 0 for l < |spin| (those coefficients do not
 *            exist, Sec. III-B); the inverse ignores them.  With reality = 1 the
 *            forward writes all L*L entries (negative m by the symmetry of
 *            Sec. IV-G) and the inverse reads only m >= 0.
 *
 * Batches: every per-map argument (L, spin, reality) is a HOST array of length
 * `batch`; `ptrs` is a HOST array of 2*batch DEVICE pointers, ptrs[2b] = input
 * of map b and ptrs[2b+1] = its output.  Inputs are not modified; input and
 * output of one map must not overlap.
 *
 * Streams: every call enqueues its kernels on `stream` (a hipStream_t; NULL =
 * the default stream) and returns without synchronising.  Device faults
 * surface at the caller's next synchronisation.  Calls are thread-safe.
 *
 * Precision (applies to the O(L^3) contraction only; every other stage, and the
 * Wigner recursion, always runs in FP64):
 *   MW_FP64  : FP64 throughout.  Matches a plain FP64 evaluation of the paper's
 *              algorithms to <= 1e-12 (infinity-norm relative error).
 *   MW_FP32C : the FP64 Wigner products Delta*Delta and the Fourier data are
 *              rounded to FP32 and accumulated in FP32 on the matrix cores over
 *              segments of the chains, the segments being added in FP64.  Maps
 *              of one spin in a call share the FP64 recursions.  Stated accuracy:
 *              <= 1e-6 infinity-norm relative error against FP64.
 *
 * Errors: arguments are validated before anything is enqueued.  Return values
 * are mw_status codes; mw_status_string() gives a description, and
 * mw_last_error() the detail of the last failure in this thread.
 *
 * Memory: the library owns per-band-limit plan tables and a workspace for
 * intermediates, both allocated on first use on the current device (outside any
 * stream capture) and kept until mw_release() or process exit.  A caller may
 * instead bind a workspace of its own to a stream (mw_set_workspace).  The
 * library never frees caller memory.
 * ---------------------------------------------------------------------------
 */
#ifndef MW_H
#define MW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MW_OK = 0,
    MW_EINVAL = -1,   /* invalid argument (see validation rules below)            */
    MW_ENOMEM = -2,   /* device or host allocation failed                         */
    MW_EHIP = -3,     /* a HIP runtime call or kernel launch failed               */
    MW_ENOTSUP = -4   /* valid request that this build does not support           */
} mw_status;

typedef enum {
    MW_FP64 = 0,
    MW_FP32C = 1
} mw_precision;

/* Largest band-limit: the Wigner recursions stay accurate to l = 4095 with their
 * exponent-extended start values, the stability range the paper reports for its
 * own recursion (Sec. V-C, V-D). */
#define MW_LMAX 4096

/* Validation rules shared by all transform entry points (MW_EINVAL otherwise):
 *   1 <= batch;  for every map b: 1 <= L[b] <= MW_LMAX, |spin[b]| < L[b],
 *   reality[b] in {0, 1}, reality[b] = 1 only with spin[b] = 0 (the real-signal
 *   saving of Sec. IV-G is for scalar maps), ptrs and ptrs[0..2*batch-1] non-NULL,
 *   precision one of mw_precision. */

/* Forward transform (Sec. IV-D): ptrs[2b] = map, ptrs[2b+1] = coeffs. */
int mw_forward(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
               void* const* ptrs, int32_t precision, void* stream);

/* Forward transform that allocates nothing, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, layouts and results as mw_forward (the
 * same kernels, bit for bit), but the intermediates live in a static device
 * array of MW_NOALLOC_BYTES that every device the library runs on holds from
 * the library's load until the process ends; the call makes no hipMalloc,
 * hipFree or other allocation, creates no stream or event, and runs all of its
 * maps on `stream` (no internal streams).
 *   - The plan tables must exist: call mw_prepare with the same arguments once
 *     beforehand, else MW_ENOMEM before anything is enqueued.
 *   - Limit: the workspace of the call (one set of slots for the largest chunk
 *     of equal (L, spin, reality); about 25 MB per map at L = 512, 6.3 MB at
 *     L = 256) must fit MW_NOALLOC_BYTES, else MW_ENOMEM before anything is
 *     enqueued (mw_last_error gives both sizes).
 *   - Every call on one device shares that device's array, which keeps the last
 *     call's intermediates (nothing in it needs to start at zero).  Calls that
 *     overlap on one device (different streams, or graph replays in flight)
 *     race on it: the caller must order them. */
#define MW_NOALLOC_BYTES ((size_t)64 << 20)
int mw_forward_noalloc(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                       void* const* ptrs, int32_t precision, void* stream);

/* Inverse transform (Sec. IV-E): ptrs[2b] = coeffs, ptrs[2b+1] = map. */
int mw_inverse(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
               void* const* ptrs, int32_t precision, void* stream);

/* Adjoint (conjugate transpose) of the forward map with respect to the Euclidean
 * inner products on the full L x (2L-1) grid and on the L*L coefficients: the
 * forward's stages (Sec. IV-D) transposed and conjugated in reverse order, i.e.
 * contraction^H (= the inverse's contraction, Eq.(Fmm)), unfold, correlation with
 * the conjugate weights (Eq.(Gmm_convolution)^H), positive-exponent theta DFT over
 * the whole period (Eq.(Gmm)^H), fold of the periodic extension back onto
 * t < L (Eq.(Gmt)^H) and (2 pi/N1) x the inverse phi DFT (Eq.(Gmt)^H).  It is not
 * the inverse transform.  ptrs[2b] = coeffs-space input (complex128, all L*L
 * entries used, entries with l < |spin| ignored), ptrs[2b+1] = map-space output.
 * With reality = 1 the output is the float64 map Re(A^H y), the adjoint of the
 * forward restricted to real maps.  This is the reverse-mode derivative of
 * mw_forward: for a real loss, grad_map = A^H grad_coeffs. */
int mw_forward_adjoint(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                       void* const* ptrs, int32_t precision, void* stream);

/* Adjoint of the inverse map (Sec. IV-E transposed): Y^H g = contraction^H of
 * Z_{m m'} = sum_{t<L} e^{-i m' theta_t} sum_p e^{-i m phi_p} g(t, p), where the
 * contraction^H is the forward's Eq.(flm_wig) with the fold of Eq.(Fmm_sym1)
 * (no weights, no extension, no 1/(2 pi N1)).  ptrs[2b] = map-space input,
 * ptrs[2b+1] = coeffs-space output (complex128, L*L entries, 0 for l < |spin|).
 * With reality = 1 the input is a float64 map and the output is the adjoint of
 * the real inverse (which reads only m >= 0): y_{l,m} + (-1)^m conj(y_{l,-m})
 * for m > 0, y_{l,0} unchanged, and 0 for m < 0. */
int mw_inverse_adjoint(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                       void* const* ptrs, int32_t precision, void* stream);

/* Compact storage (Sec. IV-C): the sampling theorem needs N_MW = (L-1)(2L-1)+1
 * samples, the south pole theta = pi being one point.  These four entry points
 * take and return maps in that layout: rings t = 0..L-2 row-major as in the
 * full layout ([t][p], 2L-1 samples each), then one sample C = f(pi, phi_0 = 0)
 * at index (L-1)(2L-1) (the full layout truncated after that sample).  The
 * pole ring of a band-limited spin-s map is C e^{i s phi_p}: at theta = pi only
 * the order m = s survives (Sec. IV-B, the footnote on the poles), and
 *   mw_forward_compact          = mw_forward of the full grid whose pole ring is
 *                                 C e^{i s phi_p} (exact for band-limited maps);
 *   mw_inverse_compact          = mw_inverse keeping the pole ring's p = 0 sample;
 *   mw_forward_adjoint_compact  = adjoint of mw_forward_compact: the full
 *                                 adjoint's rows, and sum_p e^{-i s phi_p} x(pi, phi_p)
 *                                 as the pole sample;
 *   mw_inverse_adjoint_compact  = adjoint of mw_inverse_compact: the full
 *                                 adjoint of the map with the pole sample at p = 0
 *                                 and zeros on the rest of that ring.
 * Arguments, validation, coefficient layout, batching, streams and workspace as
 * for the full-grid entry points (real maps: float64, s = 0, C real). */
int mw_forward_compact(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                       void* const* ptrs, int32_t precision, void* stream);
int mw_inverse_compact(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                       void* const* ptrs, int32_t precision, void* stream);
int mw_forward_adjoint_compact(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                               void* const* ptrs, int32_t precision, void* stream);
int mw_inverse_adjoint_compact(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                               void* const* ptrs, int32_t precision, void* stream);

/* Spin -s coefficients for free (Sec. IV-G): if a map f of spin s has
 * coefficients sf_lm, its conjugate conj(f) is a map of spin -s with
 * coefficients (-1)^{s+m} conj(sf_{l,-m}).  Under the paper's reality condition
 * for spin signals, (sf)* = (-s)f, these are the spin -s coefficients of the
 * same signal, so a spin-s transform yields the spin -s one without a second
 * transform.  ptrs[2b] = spin[b] coefficients (complex128, L[b]^2 entries),
 * ptrs[2b+1] = the spin -spin[b] coefficients (may be the same buffer: every
 * pair (l, +-m) is read before it is written); entries with l < |spin[b]| are
 * written as 0.  Exact (sign changes and conjugation only).  Validation:
 * batch >= 1, 1 <= L[b] <= MW_LMAX, |spin[b]| < L[b], non-NULL pointers, else
 * MW_EINVAL.  Enqueued on `stream`; allocates nothing. */
int mw_spin_flip(const int32_t* L, const int32_t* spin, int32_t batch, void* const* ptrs, void* stream);

/* Explicit quadrature (Sec. IV-F, Eq.(quadrature)): the weights
 *   q(theta_t) = (2 pi/L) [wt(theta_t) + (1 - delta_{t,L-1}) (-1)^s wt(theta_{2L-2-t})],
 *   wt(theta_t) = 1/(2L-1) sum_{m'=-(L-1)}^{L-1} w(-m') e^{i m' theta_t},
 * t < L, with the weights w of the theta convolution (Sec. IV-D), written to the
 * DEVICE array q (L doubles).  Validation as for the transforms (1 <= L <=
 * MW_LMAX, |spin| < L, q non-NULL), else MW_EINVAL.  Enqueued on `stream`. */
int mw_quadrature_weights(int32_t L, int32_t spin, double* q, void* stream);

/* Sampling grids of mw_integrate. */
#define MW_GRID_QUADRATURE 0   /* the rule's grid: L rings of L samples, phi'_p = 2 pi p/L */
#define MW_GRID_TRANSFORM 1    /* the transforms' grid: L rings of 2L-1 samples */

/* Integral over the sphere of each map of a batch by the explicit quadrature
 * (Sec. IV-F): I = sum_{t<L} sum_{p<nphi} f(theta_t, 2 pi p/nphi) q(theta_t) L/nphi,
 * exact for maps band-limited at L (for nphi = L this is Eq.(quadrature) itself;
 * on the transform grid, nphi = 2L-1, the phi sum is the same exact phi
 * integral of a band-limited ring).  ptrs[2b] = map, row-major [t][p] with
 * nphi = L (MW_GRID_QUADRATURE) or 2L-1 (MW_GRID_TRANSFORM) samples per ring,
 * complex128, or float64 when reality = 1; ptrs[2b+1] = one complex128, I.
 * For spin maps the integral is that of the spin-s function as sampled.
 * Validation as for the transforms (precision does not apply), grid one of the
 * two values above, else MW_EINVAL.  Uses batch x L x 16 bytes of the workspace
 * (the library's, or one bound with mw_set_workspace); enqueued on `stream`;
 * the sums run in a fixed order (results do not depend on scheduling). */
int mw_integrate(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch, void* const* ptrs,
                 int32_t grid, void* stream);

/* Bytes of workspace one call with these arguments needs (plan tables excluded).
 * A call whose maps form several chunks (see mw_prepare) runs them alternately
 * on two internal streams, each with its own half of the workspace. */
int mw_workspace_size(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                      int32_t precision, size_t* bytes);

/* Bind a caller-owned DEVICE buffer of `bytes` bytes (dptr, 256-byte alignment
 * not required) as the workspace of every later call on `stream` (a hipStream_t;
 * NULL = the default stream) on the current device; dptr = NULL unbinds it, and
 * calls on that stream use the library's workspace again.  A bound call never
 * allocates or touches the library's workspace: if the call needs more than
 * `bytes` (mw_workspace_size with the same arguments) it fails with MW_ENOMEM
 * before enqueueing anything.  Calls on different streams with buffers of their
 * own may therefore run concurrently.  Plan tables are still the library's:
 * under stream capture, prepare them first (mw_prepare).  The buffer's contents
 * on entry do not matter; the caller keeps ownership and must keep it allocated
 * until every call (or captured graph replay) that used it has completed.
 * Enqueues nothing and does not synchronise.  MW_EINVAL for dptr != NULL with
 * bytes = 0. */
int mw_set_workspace(void* dptr, size_t bytes, void* stream);

/* Create the plan tables and workspace a call with these arguments needs, on the
 * current device, so that a later call (e.g. one under stream capture) performs
 * no allocation.  With precision MW_FP32C it also times the candidate group
 * sizes of the shared-recursion contraction for each (L, reality) class of the
 * batch and keeps the fastest for later calls of the same shape (the results do
 * not depend on the choice).  Synchronises the device.
 *
 * Batching: an FP64 call runs its maps in chunks of equal (L, spin, reality); an
 * MW_FP32C call in chunks of equal reality whose maps share the Wigner
 * recursions in groups of up to eight maps (the size tuned here per band-limit
 * and reality) with at most two different |s| (Sec. V's remark that the Wigner
 * values need not be recomputed): groups of one band-limit, except that the
 * maps of a band-limit with fewer maps in the call than the largest group join
 * the last group of a larger one (its recursions run to its largest
 * band-limit; each map masks the degrees beyond its own).  A real map alone in
 * its chunk takes the FP64 inverse contraction (its result is then the FP64
 * one, within the MW_FP32C bound a fortiori).  Each stage
 * of a chunk is one kernel launch per band-limit over its maps (the
 * contractions: one per group band-limit and set of spin rows).  Several chunks
 * alternate over two internal streams (created here or on the first such call)
 * that fork from and join back into the caller's stream; calls under
 * stream capture (hipGraph) record those launches with their arguments and
 * replay them unchanged.  Call mw_prepare with the same arguments first: a call
 * under capture that would need an allocation fails with MW_ENOMEM, before it
 * enqueues anything (the capture stays usable).  Workspaces
 * outgrown by later calls stay allocated until mw_release, so a captured graph
 * stays valid until then; concurrent calls (or replays) on one device share the
 * workspace and must be ordered by the caller. */
int mw_prepare(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
               int32_t precision);

/* Free every plan and workspace of the library (all devices), which also
 * invalidates graphs captured from library calls.  Synchronises. */
int mw_release(void);

/* Static description of a status code. */
const char* mw_status_string(int status);

/* Detail of the last failing call in this thread ("" if none). */
const char* mw_last_error(void);

/* Library version string. */
const char* mw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MW_H */
