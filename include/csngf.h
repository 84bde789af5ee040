/*
 * csngf.h - C ABI of the MI355X (gfx950) Cross-Sim-NGF hot path.
 *
 * Given a fixed volume A and a moving volume B, the library scores candidate 3-D rotations
 * of B.  For each rotation it resamples B, takes its normalized gradient field, and computes
 * the masked squared-NGF cross similarity CSNGF(chi) at EVERY integer displacement chi
 * (Sec. 3.1, Eq. (5)), using the six separable products of Eq. (6) correlated in the
 * frequency domain against A's precomputed spectra (Eq. (7)-(8)), exact integer overlap
 * counts N(chi), the minimum-overlap rule gamma (Sec. 3.2) and a per-rotation argmax.
 * The overall best (score, rotation, displacement) is the alignment (Sec. 3.2, Fig. 1).
 *
 * Conventions shared by every call
 *   - Volumes are float32, C order [nz][ny][nx] (x fastest); masks are uint8 (0 = outside)
 *     in the same layout.  Each extent must be >= 3.
 *   - Coordinates and 3x3 matrices use (x, y, z) order; matrices are row-major doubles.
 *   - A rotation R maps an output voxel x on B's grid to the source point
 *     p = R (x - c) + c in B, c = (n_B - 1) / 2 (inverse mapping: B^ = B o T_R, Sec. 3.2).
 *     Entries are rounded to multiples of 2^-16 (ties to even) before use, and must satisfy
 *     |R_ij| <= 2; the rounded matrix is what the results refer to.
 *   - B^ is sampled by trilinear interpolation; a voxel of B^ is valid when p lies in the
 *     closed box [0, n_B - 1] (and, with a mask on B, all 8 corners of its source cell are
 *     inside the mask).  NGF (Eq. (1), eps from the params) uses central differences with
 *     unit spacing; masks are eroded by the 7-point stencil so every counted voxel has all
 *     six neighbours.
 *   - A displacement chi = (chi_x, chi_y, chi_z) pairs A(x) with B^(x + chi); each component
 *     lies in [-(n_A - 1), n_B - 1].  chi is valid when N(chi) >= 1 and
 *     N(chi) >= gamma * min(|M_A|, |M_B^|).  The score is C(chi) = S(chi) / N(chi).
 *   - Ties: the larger score wins; equal scores go to the smaller canonical index
 *     (chi_z, chi_y, chi_x lexicographic, ascending); across rotations the smaller rotation
 *     index wins.
 *
 * Errors: every call returns CSNGF_OK (0) or a negative code, leaves its outputs untouched
 * on error, and records a message readable with csngf_last_error() on the same thread.
 * No exception or abort crosses the ABI.  One host thread at a time may use a context;
 * distinct contexts are independent.
 */
#ifndef CSNGF_H
#define CSNGF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSNGF_OK 0
#define CSNGF_E_INVALID_ARG (-1)    /* NULL pointer, extent < 3, non-finite input, bad gamma/eps/R */
#define CSNGF_E_UNSUPPORTED (-2)    /* FFT size not built (see csngf_supported_length), volume too large */
#define CSNGF_E_NO_DEVICE (-3)      /* no HIP device visible */
#define CSNGF_E_OUT_OF_MEMORY (-4)  /* device allocation failed */
#define CSNGF_E_DEVICE (-5)         /* HIP runtime error; message holds the HIP error text */
#define CSNGF_E_NO_VALID_SHIFT (-6) /* no displacement met gamma for any rotation; best.score = -inf */

/* params.flags: volumes, masks and map outputs are device pointers; the call is then
 * stream-ordered on the context's stream and those buffers must stay alive until the
 * stream has passed it.  Without the flag they are host pointers and calls are
 * synchronous.  Rotation matrices and result structs are always host memory. */
#define CSNGF_DEVICE_PTRS 1u
/* params.flags: score with the unsquared similarity <n_A, n_B> (Eq. (3); the USNGF variant of
 * Sec. 5.1) instead of the squared one of Eq. (2).  Its separable parts are the 3 NGF
 * components (weight 1) instead of the 6 products of Eq. (6); scores lie in [-1, 1] and
 * change sign with the gradient sign of either volume. */
#define CSNGF_UNSQUARED 2u
/* params.flags: record each context's per-batch launch sequence once as a HIP graph and
 * replay it for every full batch of rotations (re-recorded when B's device pointers change;
 * ignored while profiling is enabled).  Results are identical to the eager launches. */
#define CSNGF_GRAPHS 4u

/* params.flags: correlate the product fields in FP64 instead of FP32.  The NGF and its products
 * are the same FP32 values; the zero-padded transforms, the frequency-domain sum against A's
 * (then FP64) spectra and the inverse run in double precision, so the error of S(chi) is the
 * FP32 rounding of the products alone.  The FP32 path's S carries an absolute transform error
 * that grows with the fields' total energy (about 1e-4 on ~20^3 volumes): C = S / N meets
 * 1e-4 wherever the minimum overlap keeps N large (gamma = 0.5: N is half a mask), but not at
 * overlaps of a few voxels, which only gamma near 0 admits.  Use this flag there.  It moves
 * twice the bytes and runs the transforms at the FP64 rate. */
#define CSNGF_FP64 8u

typedef struct csngf_ctx csngf_ctx;

typedef struct {
  int32_t nx, ny, nz;
} csngf_dims;

typedef struct {
  uint32_t struct_size; /* sizeof(csngf_params) (48 bytes) */
  float eps;            /* NGF regulariser, Eq. (1); default 1e-5 */
  double gamma;         /* minimum overlap fraction in [0, 1], Sec. 3.2; default 0.5.  chi is
                           valid iff N >= 1 and N >= gamma * m with m = min(|M_A|, |M_B^|), the
                           product gamma * m taken in double precision (round to nearest), so
                           a decimal gamma such as 0.3 keeps its meaning at N = 0.3 m */
  int32_t pad[3];       /* FFT size (Px, Py, Pz); 0 = automatic: the smallest supported length
                           >= n_A + n_B - 1, or the smallest one with a compile-time plan when
                           that is at most 1.5x as long (see csngf_footprint for the result) */
  int32_t batch;        /* rotations in flight per launch sequence, 0 .. 255; 0 = automatic */
  uint32_t flags;       /* CSNGF_DEVICE_PTRS | CSNGF_UNSQUARED | CSNGF_GRAPHS | CSNGF_FP64 */
  int32_t slices;       /* z slices per field-stage workgroup, 0 .. 64; 0 = automatic (8).  More
                           slices re-sample fewer halo planes, fewer give more workgroups */
  int32_t final_groups; /* workgroups of the final pass when no map is written, 0 .. 65535;
                           0 = automatic (8192); they walk the list of row groups that hold a
                           valid displacement */
  int32_t reserved;     /* must be 0 */
} csngf_params;

typedef struct {
  float score;      /* C at the argmax; -inf when no displacement is valid */
  int32_t shift[3]; /* argmax displacement (chi_x, chi_y, chi_z) */
  int64_t overlap;  /* N at the argmax (exact) */
  int32_t valid;    /* 1 when some displacement met gamma */
  int32_t reserved;
} csngf_rot_result;

typedef struct {
  float score;      /* best C over all rotations; -inf when none is valid */
  int32_t rot_index;/* index into the rotation array; -1 when none is valid */
  int32_t shift[3];
  int32_t reserved;
  int64_t overlap;
  double R[9];      /* the quantised matrix actually used */
} csngf_best;

typedef struct {
  int32_t pad[3];          /* FFT size in use (Px, Py, Pz) */
  int32_t batch;           /* rotation slots in flight */
  int32_t map_dims[3];     /* W = n_A + n_B - 1 per axis (x, y, z) */
  int32_t reserved;
  int64_t count_a;         /* |M_A| after erosion */
  int64_t spectra_bytes;   /* device bytes held per context: A's conjugate spectra and the
                              moving volume's brick copy (5^3 values per 4^3 cells) */
  int64_t workspace_bytes; /* device bytes held for rotation workspaces */
} csngf_info;

/* Fill *out with the defaults (eps 1e-5, gamma 0.5, automatic padding and batch). */
int csngf_default_params(csngf_params* out);

/* 1 when an FFT of length L is built into the library (L even, 8 <= L <= 512, only prime
 * factors 2, 3, 5, 7, 11), else 0. */
int csngf_supported_length(int32_t L);

/* Precompute the fixed side for volume A (dims dA) against moving volumes of dims dB:
 * NGF of A, its six weighted product fields (cross terms x2, Eq. (6)), their zero-padded
 * 3-D FFTs, conjugated and kept resident on the device (Sec. 3.1, Eq. (7)-(8)).
 * maskA: NULL = full domain (eroded to the box [1, n_A - 2]), or a uint8 mask M_A in A's
 * layout (nonzero = inside; Sec. 3.1, Eq. (4)-(5)), eroded like B's so every counted voxel
 * has its six neighbours.  With NULL, N(chi) is an integer box sum over B^'s mask.  With a
 * mask, N(chi) is the mask cross-correlation of Sec. 3.1 (after Eq. (5)), computed by FP64
 * zero-padded FFTs against A's resident FP64 mask spectrum and rounded to the exact integer
 * (the FP64 error is far below 1/2); this adds one FP64 pencil chain per rotation and about
 * 16 B x (2 W_z P_y + W_z W_y) x Px/2 + 4 B x W_x W_y W_z of workspace per rotation slot (the
 * figure csngf_footprint reports is for NULL; csngf_get_info gives the context's own).
 * A and maskA are copied; the caller may free them on return.  p may be NULL for the
 * defaults.  On success *out owns all device memory. */
int csngf_create(const float* A, csngf_dims dA, const uint8_t* maskA, csngf_dims dB,
                 const csngf_params* p, csngf_ctx** out);

/* Use the given hipStream_t (e.g. PyTorch's current stream) for all later work; NULL
 * restores the context's own stream.  The caller keeps ownership of the stream.  Part of
 * each evaluation (the overlap table and a few FFT tiles) runs on a second stream that the
 * context owns; it forks from and joins back into this stream with events, so all work of a
 * call is ordered on this stream as seen from outside, also under graph capture. */
int csngf_set_stream(csngf_ctx* ctx, void* hip_stream);

int csngf_get_info(const csngf_ctx* ctx, csngf_info* out);

/* Score n rotations (R: n x 9 row-major doubles, host) of moving volume B (dims dB of the
 * context; maskB NULL = full domain): for each rotation, B resampled under it (Sec. 3.2),
 * C(chi) of Sec. 3.1, Eq. (5) at every displacement chi via Eq. (6)-(8), and the argmax over
 * the chi that meet the minimum overlap (Sec. 3.2); best = the largest over rotations, the
 * alignment of Sec. 3.2.  per_rot (host, n entries) may be NULL; best (host) may be NULL.
 * Returns CSNGF_E_NO_VALID_SHIFT when no rotation has a valid displacement (per_rot still
 * filled).  n == 0 is valid: best->rot_index = -1. */
int csngf_evaluate(csngf_ctx* ctx, const float* B, const uint8_t* maskB, const double* R,
                   int32_t n, csngf_rot_result* per_rot, csngf_best* best);

/* Asynchronous form of csngf_evaluate: validates and quantises the rotations, enqueues the
 * whole evaluation on the context's stream and returns.  B and maskB must stay valid until
 * csngf_wait returns.  One evaluation may be in flight per context; contexts on different
 * streams run concurrently on the device (many volume pairs at once). */
int csngf_evaluate_async(csngf_ctx* ctx, const float* B, const uint8_t* maskB, const double* R, int32_t n);

/* 1 when the context has no evaluation in flight or it has finished, 0 while it runs. */
int csngf_query(csngf_ctx* ctx);

/* Wait for the evaluation in flight and return its results exactly as csngf_evaluate would
 * (per_rot: n entries or NULL; best or NULL).  CSNGF_E_INVALID_ARG when none is in flight. */
int csngf_wait(csngf_ctx* ctx, csngf_rot_result* per_rot, csngf_best* best);

/* Full maps for one rotation (diagnosis and parity): C(chi) of Sec. 3.1, Eq. (5) as
 * C[Wz][Wy][Wx] float32 with -inf where chi misses the minimum overlap of Sec. 3.2, and
 * optionally the overlap counts N(chi) (Sec. 3.1, after Eq. (5)) as N[Wz][Wy][Wx] int64 (may be
 * NULL).  Index i = chi + n_A - 1 per axis.  Host or device pointers per params.flags. */
int csngf_evaluate_map(csngf_ctx* ctx, const float* B, const uint8_t* maskB, const double* R9,
                       float* C, int64_t* N);

int csngf_destroy(csngf_ctx* ctx);

/* One level of the Gaussian pyramid of the global search (Sec. 3.2): blur vol (dims d) with
 * a Gaussian of standard deviation sigma voxels per axis (taps exp(-k^2 / (2 sigma^2)) for
 * |k| <= int(4 sigma + 0.5), normalised to sum 1, edge samples replicated; sigma = 0 copies)
 * and keep every factor-th voxel from index 0: out dims m = ceil(n / factor) per axis,
 * out[z][y][x] = blurred[factor z][factor y][factor x].  *out_dims receives m (may be
 * queried with out = NULL).  Device pointers with CSNGF_DEVICE_PTRS in flags (asynchronous
 * on stream), host pointers otherwise (synchronous).  factor >= 1, sigma in [0, 64]. */
int csngf_smooth_downsample(const float* vol, csngf_dims d, float sigma, int32_t factor, float* out,
                            csngf_dims* out_dims, uint32_t flags, void* stream);

/* Allocation-free form of csngf_smooth_downsample, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments and bit-identical results, but vol and out are always DEVICE pointers on the
 * current device, and the call only enqueues the blur on stream (a hipStream_t; NULL = the
 * default stream) and returns; no hipMalloc, hipFree or other allocating call is made.
 * The two intermediate volumes of the separable blur (m0 n1 n2 and m0 m1 n2 floats, n = dims
 * d, m = out dims) live in a fixed scratch array of CSNGF_NOALLOC_SCRATCH_BYTES that the
 * library holds on each device it runs on until the process ends; inputs whose intermediates
 * do not fit return CSNGF_E_UNSUPPORTED.  Every call on a device shares that device's array,
 * so calls that overlap in time on one device race: order them (one stream, or events).
 * The array is fully written before it is read, so nothing is left over from earlier calls. */
#define CSNGF_NOALLOC_SCRATCH_BYTES (32u << 20)
int csngf_smooth_downsample_noalloc(const float* vol, csngf_dims d, float sigma, int32_t factor, float* out,
                                    csngf_dims* out_dims, void* stream);

/* Device memory a context would hold, without allocating anything (admission control of a
 * server): *spectra_bytes per context (A's resident spectra and B's brick copy),
 * *slot_bytes per rotation slot of workspace (a context holds batch slots), and the FFT size
 * pad_out[3] that would be used.
 * Any output may be NULL. */
int csngf_footprint(csngf_dims dA, csngf_dims dB, const csngf_params* p, int64_t* spectra_bytes,
                    int64_t* slot_bytes, int32_t* pad_out);

/* Autotuner: for the shapes of A and B and the base params (eps, gamma, flags), time the
 * candidate configurations - FFT size per axis (the smallest supported length and the next
 * length with a compile-time plan within 1.5x, every combination, with the automatic slot
 * count), then at the best size the rotation slots in flight (half and double), then z
 * slices per field-stage workgroup (4, 8, 16) and then final-pass workgroups (2048 .. 16384) - on
 * n_probe deterministic random rotations, and return the fastest in *best (pad, batch,
 * slices and final_groups set) and its rate in rotations/s (*best_rate may be NULL).  Creates
 * and destroys contexts; results do not depend on the choice (any FFT size >= n_A + n_B - 1
 * gives the same linear correlation, and the launch shapes only split the same work). */
int csngf_autotune(const float* A, csngf_dims dA, const float* B, csngf_dims dB, const csngf_params* base,
                   int32_t n_probe, csngf_params* best, double* best_rate);

/* Message of the last failed call on this thread ("" if none). */
const char* csngf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CSNGF_H */
