/*
 * pat.h -- C ABI of the MI355X (gfx950) photoacoustic-tomography hot path.
 *
 * Method: Arridge, Beard, Betcke, Cox, Huynh, Lucka, Ogunlade, Zhang,
 * "Accelerated high-resolution photoacoustic tomography via compressed
 * sensing" (arXiv 1605.00133). The library computes
 *
 *   f = C A p0                     measurement model, eq. (Fwd), Sec. 4.1
 *   p = A^T C^T f                  back-projection / gradient, eq. (BP), Sec. 4.4
 *   q = prox_{TV + (q>=0), alpha}  positivity-constrained TV denoising, eq. (Prox), App. A/B
 *   p = argmin 1/2||CAp - f||^2 + lambda TV(p), p >= 0   eq. (VarReg)/(TV+), by FISTA (App. B)
 *       optionally enhanced by Bregman iterations, eq. (BregIterA/B), Sec. 4.6
 *
 * where A is 3D linear acoustic propagation of the initial pressure
 * (eq. PATfwd) by a k-space pseudospectral scheme with a perfectly matched
 * layer, sampled on the detection plane z = 0 at every time step (Sec. 4.3),
 * and C is the sub-sampling operator: every plane pixel, random single
 * points (rSP) or scrambled +-1 Hadamard patterns (sHd) (Sec. 3.1, 4.3).
 *
 * Conventions shared by every entry point
 *  - Volumes are float32 arrays [nz][ny][nx] (x fastest); the detection plane
 *    is the slab z = 0. Data arrays are float32 [nt][mc] (time-major).
 *  - Pointers named "device" are HIP device pointers; all other pointers are
 *    host pointers. The caller owns every buffer it passes; the library never
 *    frees caller memory.
 *  - Work is enqueued asynchronously on the plan's HIP stream unless the entry
 *    point returns a host value (those synchronise the stream).
 *  - Every call returns a pat_status and never aborts; pat_last_error() gives
 *    a message for the last non-OK status of the calling thread. Arguments
 *    are validated before any work is enqueued.
 *  - Results are deterministic: no floating-point atomics, fixed reduction
 *    trees (FP64 partial sums for every reported scalar).
 *  - Concurrent calls on one plan are not allowed (the plan's workspace is
 *    shared by all its entry points); distinct plans are independent.
 */
#ifndef PAT_H
#define PAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PAT_OK = 0,
  PAT_ERR_INVALID = 1,      /* bad argument: null pointer, size, range */
  PAT_ERR_UNSUPPORTED = 2,  /* valid but not built: grid size, non power-of-two Hadamard plane */
  PAT_ERR_NOMEM = 3,        /* workspace too small or a table allocation failed */
  PAT_ERR_HIP = 4,          /* HIP runtime or launch error */
  PAT_ERR_NONFINITE = 5     /* a reported scalar is NaN or Inf */
} pat_status;

/* Discretisation (Table 2 lists the paper's values). The FFT grid includes
 * the PML: pml_size cells on each side in x and y, and a 2*pml_size slab at
 * the top of z (z in [nz - 2 pml, nz)), so the plane z = 0 sits directly in
 * front of it. The grid is cubic, nx = ny = nz one of the built sizes (16, 32,
 * 64, 96, 128; 96 uses radix-3 butterflies), and nt >= 1. */
typedef struct {
  int32_t nx, ny, nz;
  double dx;          /* voxel size [m], isotropic */
  double c0;          /* homogeneous sound speed [m/s] */
  double rho0;        /* ambient density; A does not depend on it (> 0) */
  double dt;          /* time step = temporal sampling interval [s] */
  int32_t nt;         /* samples at t = 0, dt, ..., (nt-1) dt */
  int32_t pml_size;   /* P >= 0, 2P < min(nx, ny) and 2P < nz */
  double pml_alpha;   /* absorption sigma = alpha (c0/dx) d^4, d in [0,1] */
} pat_grid;

typedef enum {
  PAT_SAMPLE_FULL = 0,      /* conventional scan: every plane pixel, mc = nx*ny */
  PAT_SAMPLE_POINTS = 1,    /* rSP: idx = mc sorted distinct pixel ids iy*nx+ix */
  PAT_SAMPLE_HADAMARD = 2   /* sHd: f_j = (W x~)[idx_j] / sqrt(nx*ny), x~[q] = s[perm[q]] */
} pat_sample_kind;

/* Sub-sampling operator C (Sec. 3.1, 4.3). idx and perm are HOST arrays and
 * are copied into the plan. POINTS: idx[mc] strictly increasing in
 * [0, nx*ny). HADAMARD: nx*ny a power of two, perm[nx*ny] a permutation,
 * idx[mc] strictly increasing Sylvester-Walsh row ids. C C^T = I for all kinds. */
typedef struct {
  int32_t kind;               /* pat_sample_kind */
  int32_t mc;                 /* rows of f per time step */
  const int32_t* idx;         /* host; NULL for FULL */
  const int32_t* perm;        /* host; HADAMARD only */
} pat_sampling;

typedef struct pat_plan pat_plan;

/* Bytes of device workspace a plan needs (state fields, spectra, the plane
 * time series and the solver vectors). Returns 0 for invalid arguments. */
size_t pat_plan_workspace_bytes(const pat_grid* grid, const pat_sampling* smp);

/* Create a plan: validates grid and sampling, uploads the small tables
 * (twiddles, wavenumbers, PML factors, index maps) and carves `workspace`
 * (device, >= pat_plan_workspace_bytes, 256-byte aligned, caller-owned and
 * kept alive until pat_plan_destroy). stream: a hipStream_t or NULL. */
pat_status pat_plan_create(const pat_grid* grid, const pat_sampling* smp, void* stream,
                           void* workspace, size_t workspace_bytes, pat_plan** out);
pat_status pat_plan_destroy(pat_plan* plan);
pat_status pat_plan_set_stream(pat_plan* plan, void* stream);

/* Spatially varying sensor sensitivity W_s (eq. FwdSenVar, Sec. 5.3): with a
 * weight per pixel of the detection plane, pat_forward computes C W_s A p0 (each
 * pixel's pressure time course scaled by its weight before sub-sampling) and
 * pat_adjoint A^T W_s C^T f, so the pair stay exact transposes. w: HOST array of
 * nx*ny finite floats [iy][ix], copied into a device buffer the plan owns (one
 * allocation on the first call); NULL restores the ideal sensor. Used to
 * generate data with a model other than the one reconstructed with. */
pat_status pat_plan_set_sensitivity(pat_plan* plan, const float* w);

/* A heterogeneous medium for data generation (the sound-speed perturbation of
 * the no-inverse-crime data, Sec. 5.3): c is a HOST array of nz*ny*nx speeds
 * [z][y][x], each positive and at most the grid's c0, which becomes the reference
 * speed of the k-space correction (and of the CFL number). pat_forward then
 * computes the pressure as c(x)^2 times the summed densities, with initial
 * densities p0 / (3 c(x)^2), on the slab scheme whatever the plan's scheme.
 * pat_adjoint, pat_time_reversal and pat_reconstruct need the homogeneous medium
 * and return PAT_ERR_UNSUPPORTED while a field is set; NULL clears it. The field
 * is copied into a device buffer the plan owns (allocated on the first call). */
pat_status pat_plan_set_sound_speed(pat_plan* plan, const float* c);

/* Arithmetic of the propagator's FFT butterflies: 64 (default) keeps FP64
 * values in registers and LDS inside each transform pass and rounds to FP32
 * once per pass; 32 computes in FP32 throughout (faster, about 5x larger
 * rounding error, which accumulates over the Nt time steps). Stored fields
 * and spectra are FP32 in both cases. */
pat_status pat_plan_set_fft_precision(pat_plan* plan, int32_t bits);

/* Which implementation of the propagator A, A^T (Sec. 4.3) the plan runs;
 * both compute the same operator.
 *  PAT_SCHEME_SLAB: per time step, 2D slab transforms fused with the state
 *    updates and z-pencil passes fused with the k-space multipliers;
 *  PAT_SCHEME_LINE (default where built: cubic grids): every field component
 *    kept real along its own axis and transformed along the other two, so a
 *    time step is one launch of independent 1D lines (four transforms per
 *    line). It needs FP64 butterflies; with pat_plan_set_fft_precision(32)
 *    the slab scheme runs. Returns PAT_ERR_UNSUPPORTED when the grid has no
 *    line propagator.
 * Only the line scheme may be captured into a HIP graph: the slab scheme's
 * hand-off flags are tagged with a per-launch count kept on the host, so its
 * operator calls return PAT_ERR_UNSUPPORTED on a capturing stream. */
typedef enum { PAT_SCHEME_SLAB = 0, PAT_SCHEME_LINE = 1 } pat_scheme;
pat_status pat_plan_set_scheme(pat_plan* plan, int32_t scheme);

/* f = C A p0 (eq. Fwd without noise). p0: device [nz][ny][nx]; f: device [nt][mc].
 * p0 and f must not overlap. */
pat_status pat_forward(pat_plan* plan, const float* p0, float* f);

/* p = A^T C^T f, the exact transpose of pat_forward's arithmetic (eq. BP).
 * f: device [nt][mc]; p: device [nz][ny][nx]; no overlap. */
pat_status pat_adjoint(pat_plan* plan, const float* f, float* p);

/* p = A^< C^T f, time reversal (eq. TRnum, Sec. 4.4): the propagator run from
 * zero fields with the time-reversed series C^T f imposed on the detection plane
 * as a Dirichlet condition (at the start and after every density update, each
 * density component on z = 0 is set to the datum / (3 c0^2)); p is the pressure
 * field after the last step (its plane z = 0 is the datum at t = 0). A linear
 * two-step baseline, not an adjoint. Runs the slab scheme (real-space fields)
 * with the plan's FFT precision whatever the plan's scheme, ignores the sensor
 * sensitivity, and cannot be captured into a graph (PAT_ERR_UNSUPPORTED).
 * f: device [nt][mc]; p: device [nz][ny][nx]; no overlap. */
pat_status pat_time_reversal(pat_plan* plan, const float* f, float* p);

/* C alone on a plane series s: device [nt][ny][nx] -> f: device [nt][mc]. */
pat_status pat_sample(pat_plan* plan, const float* s, float* f);
/* C^T alone: f: device [nt][mc] -> s: device [nt][ny][nx]. */
pat_status pat_sample_adjoint(pat_plan* plan, const float* f, float* s);

/* Floats of the PDHG dual for pat_tv_prox: bc = 0 (Neumann) 3*nx*ny*nz laid
 * out [3][nz][ny][nx]; bc = 1 (Dirichlet) 3*(nx+1)*(ny+1)*(nz+1) laid out
 * [3][nz+1][ny+1][nx+1] over the zero-padded grid's points 0..n (components x, y, z). */
size_t pat_tv_dual_floats(const pat_grid* grid, int32_t bc);

/* q = argmin_{q >= 0} 1/2||q - v||^2 + alpha TV(q) by n_iter iterations of the
 * accelerated primal-dual hybrid gradient method (App. B), q started at
 * max(0, v), step sizes 1/sqrt(12). TV is isotropic forward differences with
 * Neumann (bc = 0) or Dirichlet (bc = 1, jumps to zero at the faces added)
 * boundaries (App. A). v, q: device volumes, may alias. dual: device,
 * pat_tv_dual_floats(bc) floats, in/out warm start (zero it for a cold start). */
pat_status pat_tv_prox(pat_plan* plan, const float* v, float* q, float alpha, int32_t n_iter,
                       int32_t bc, float* dual);

/* TV(p) (App. A) as an FP64 host value; syncs. */
pat_status pat_tv_norm(pat_plan* plan, const float* p, int32_t bc, double* out);

/* Largest eigenvalue of A^T C^T C A by n_iter power steps from x0 (device
 * volume, not modified): x <- x0/|x0|; repeat w = A^T C^T C A x, L = |w|,
 * x = w/L. Used for the step size eta = 1.8/L (App. B). Host result; syncs. */
pat_status pat_power_iteration(pat_plan* plan, const float* x0, int32_t n_iter, double* L_out);

typedef struct {
  double lambda;          /* TV weight */
  double L;               /* Lipschitz estimate of A^T C^T C A; eta = 1.8 / L */
  int32_t n_outer;        /* Bregman iterations (1 = plain TV+) */
  int32_t n_inner;        /* FISTA iterations per outer step */
  int32_t n_prox;         /* PDHG iterations per prox */
  int32_t bc;             /* TV boundary: 0 Neumann, 1 Dirichlet */
  int32_t restart;        /* 1: restart + backtracking on energy increase */
  int32_t max_backtrack;  /* halvings after the plain gradient step (paper: 5) */
  const float* p_ref;     /* optional device volume for PSNR logging, or NULL */
} pat_recon_params;

/* Per-FISTA-iteration log, host buffers owned by the caller, each with
 * `capacity` entries (any pointer may be NULL). Entry i is iteration i of the
 * flattened outer x inner loop. flags: 0 plain step, 1 + j restart that kept
 * the step after j halvings. residual: ||C A x - d||; energy: 1/2 residual^2 +
 * lambda TV(x); bregman_residual (per outer step): ||C A p^k - f||. */
typedef struct {
  int32_t capacity;
  int32_t n_log;          /* out: entries written */
  double* energy;
  double* residual;
  double* tv;
  int32_t* flags;
  double* psnr;           /* needs p_ref */
  double* t_ms;           /* wall time since the call started, after the iteration */
  double* bregman_residual; /* n_outer entries */
} pat_recon_report;

/* TV+ (n_outer = 1) or TV+Br reconstruction of p from f (device [nt][mc]) into p
 * (device volume; output only: the first FISTA loop starts from p = 0, whose
 * residual is -f without an operator application, and each Bregman step from
 * the previous one's result). Syncs once per FISTA iteration to read the FP64
 * energy. */
pat_status pat_reconstruct(pat_plan* plan, const float* f, float* p,
                           const pat_recon_params* params, pat_recon_report* report);

/* n_iter FISTA iterations of TV+ (eq. VarReg/TV+, App. B) from p = 0 without
 * restart, enqueued on the plan's stream with no host synchronisation and no
 * memory copies or sets (kernels only), so that the whole call can be captured
 * into a HIP graph; it is the arithmetic of pat_reconstruct with n_outer = 1
 * and restart = 0, and gives the same p bit for bit. f: device [nt][mc];
 * p: device volume (output); log: NULL or device FP64 [n_iter][2] receiving
 * sum((C A x - f)^2) and TV(x) of each iterate (the energy is half the first
 * plus lambda times the second). Arguments are checked on the host; nothing is
 * read back, so non-finite values show up only in p and the log. */
pat_status pat_fista_enqueue(pat_plan* plan, const float* f, float* p, double lambda, double L, int32_t n_iter,
                             int32_t n_prox, int32_t bc, double* log);

/* Iterations it0 .. it0 + n_iter - 1 of the same loop (eq. VarReg/TV+, App. B),
 * so that one reconstruction can be enqueued, or captured, in several parts:
 * it0 = 0 is pat_fista_enqueue; it0 > 0 continues from the iterate, its
 * predecessor, the extrapolated point, their residuals and the prox dual that
 * the call for iterations 0 .. it0 - 1 left in the plan's workspace, with the
 * same f, lambda, L, n_prox and bc. The parts together give p bit for bit as
 * one call of it0 + n_iter iterations. No other pat_reconstruct,
 * pat_fista_enqueue(_from) or pat_power_iteration call may run on the plan
 * between the parts (they use the same workspace); pat_forward, pat_adjoint and
 * pat_psnr may. log: NULL or device FP64 [n_iter][2] for these iterations.
 * p receives the latest iterate after every part. */
pat_status pat_fista_enqueue_from(pat_plan* plan, const float* f, float* p, double lambda, double L, int32_t it0,
                                  int32_t n_iter, int32_t n_prox, int32_t bc, double* log);

/* Thresholded PSNR of p against p_ref (eq. PSNR) over the non-PML interior with
 * z >= 1: negatives clipped, both scaled by their maximum, values < 0.1 zeroed.
 * p, p_ref: device volumes. Host result; syncs. +Inf when identical. */
pat_status pat_psnr(pat_plan* plan, const float* p, const float* p_ref, double* out);

/* Diagnostics: HIP-event timing of the propagator's kernels, for roofline
 * reporting. Between pat_profile_begin and pat_profile_end the launches of
 * kernel `kernel_id` (or of all of them, kernel_id = -2) made by pat_forward,
 * pat_adjoint and the solvers on this plan are bracketed by events on the
 * plan's stream: each launch by its own pair (slab scheme), or each run of
 * consecutive time steps of one application by one pair counted as that many
 * launches (line scheme: per-launch events would add their gaps to every
 * step), up to max_launches records. pat_profile_end syncs and fills
 * total_ms[PAT_K_COUNT] and launches[PAT_K_COUNT] (host, either may be NULL). */
typedef enum {
  PAT_K_ZGRAD = 0,      /* forward: z pass of the gradient (1 spectrum in, 2 out) */
  PAT_K_FWD_U = 1,      /* forward: slab pass, velocity update and its 2D FFT (per component) */
  PAT_K_ZDIV = 2,       /* forward: z pass of the divergences (per component) */
  PAT_K_FWD_RHO = 3,    /* forward: slab pass, density update, pressure, sensor plane, 2D FFT */
  PAT_K_ZGRAD_ADJ = 4,  /* adjoint: z pass of the gradients (per component) */
  PAT_K_ADJ_U = 5,      /* adjoint: slab pass, velocity update and its 2D FFT (per component) */
  PAT_K_ZDIV_SUM = 6,   /* adjoint: z pass of the summed divergence (3 in, 1 out) */
  PAT_K_ADJ_RHO = 7,    /* adjoint: slab pass, density update with the data source, 2D FFT */
  PAT_K_LINE_FWD = 8,   /* line scheme: one forward time step of all three components */
  PAT_K_LINE_ADJ = 9,   /* line scheme: one adjoint time step of all three components */
  PAT_K_COUNT = 10
} pat_kernel_id;

pat_status pat_profile_begin(pat_plan* plan, int32_t kernel_id, int32_t max_launches);
pat_status pat_profile_end(pat_plan* plan, double* total_ms, int32_t* launches);

/* Name and algorithmic HBM bytes per launch of a kernel on this plan's grid:
 * every field a launch must read or write once (slab spectra of
 * nz*(nx/2+1)*ny complex floats, real fields of nx*ny*nz floats, the sensor
 * plane). *name points to static storage. */
pat_status pat_kernel_info(const pat_plan* plan, int32_t kernel_id, const char** name, double* bytes_per_launch);

/* Diagnostics: dst = src for nbytes on `stream` (a hipStream_t; NULL: the
 * default stream) with a plain copy kernel (each block copies 16 KB of
 * consecutive 16-byte words, four loads in flight per thread): the practical
 * HBM copy rate of the device, against which the propagator's bandwidth is
 * reported. src,
 * dst: device, 16-byte aligned, not overlapping; nbytes a multiple of 16 in
 * [0, 2^40]. Asynchronous; errors of the arguments are returned at once. */
pat_status pat_copy_probe(const void* src, void* dst, int64_t nbytes, void* stream);

/* Host-only index generators (no GPU needed). SplitMix64(seed) drives a
 * Durstenfeld Fisher-Yates shuffle of [0, n_pix) with unbiased rejection draws.
 * rSP: the first mc entries, sorted ascending. sHd: perm = shuffle(seed), rows =
 * first mc entries of shuffle(seed + 1), sorted; n_pix must be a power of two. */
pat_status pat_make_rsp_mask(int32_t n_pix, int32_t mc, uint64_t seed, int32_t* idx_out);
pat_status pat_make_shd_pattern(int32_t n_pix, int32_t mc, uint64_t seed,
                                int32_t* perm_out, int32_t* rows_out);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char* pat_last_error(void);

/* Library version string. */
const char* pat_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PAT_H */
