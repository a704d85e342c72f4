/*
 * dsbt.h -- C ABI of the MI355X orthogonal discrete spherical Bessel transform.
 *
 * The operation (Serov, "Orthogonal fast spherical Bessel transform on uniform
 * grid"): for a radial channel of angular momentum l sampled on
 * r_i = (i - 1/2) dr, i = 1..N (Sec. 2.2, eq. r_grid), with psi_i = psi(r_i) sqrt(dr),
 *
 *     forward   b   = T F psi        (Sec. 2.2 eq. f_vs_psi; Sec. 2.4 eq. b_vs_f)
 *     inverse   psi = F^T T^T b      (eq. f_vs_b with T^{-1} = T^T, F^{-1} = F^T)
 *
 * F is the orthonormal sine (even l) or cosine (odd l) transform of
 * eq. csFourierBasis, T the Fourier-to-Bessel matrix built from derivatives of
 * discrete Legendre orthogonal polynomials (Sec. 2.4 eq. Tdef/Ldef) completed by
 * ceil(l/2) DLOP rows (Sec. 2.5 eq. Tadd).  Both are real and orthogonal; complex
 * data is transformed linearly.  Conventions (orthonormal F, the sign
 * (-1)^ceil(l/2) in F, numerically normalised rows) follow the readings listed
 * with the library's design notes.
 *
 * The split-operator step of Sec. 4.1 with zero vector potential,
 *
 *     psi <- exp(-i s V tau/2) F^T T^T exp(-i K tau) T F exp(-i s V tau/2) psi,
 *
 * uses the diagonal kinetic energy K_n = k_nl^2 / 2 of eq. KinMat.
 *
 * Data layout.  Every data buffer is a device pointer to packed interleaved
 * complex values (re, im) -- complex64 (float2) for DSBT_C64 and DSBT_C64_FP64
 * plans, complex128 (double2) for DSBT_C128 plans -- the same memory layout as torch.complex64 /
 * torch.complex128.  Channel c occupies elements [offset_c, offset_c + N_c).
 * Coefficient vectors b are stored in slot order j = n - p_l, n = p_l..N_l,
 * where p_l = 1 for even l and 0 for odd l (eq. k_grid).
 *
 * Ownership.  The caller owns every data buffer; the library never frees or
 * retains them past the call.  A plan owns its device tables and is released
 * by dsbt_plan_destroy.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null stream).
 * Transform and step calls only enqueue work on that stream and return; they
 * do not synchronise.  dsbt_plan_create and dsbt_set_potential synchronise.
 *
 * Errors.  Every call returns a dsbt_status; 0 is success.  No exception
 * crosses the ABI.  dsbt_last_error() gives a thread-local message for the
 * most recent failure.  A HIP error from an earlier asynchronous launch may be
 * reported by a later call as DSBT_ERR_HIP.
 *
 * Thread safety.  A plan is read-only after creation except for
 * dsbt_set_potential and the graph cache used by dsbt_kinetic_step; calls on
 * one plan from several host threads must not overlap those two.
 */
#ifndef DSBT_H
#define DSBT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dsbt_status;
enum {
    DSBT_OK = 0,
    DSBT_ERR_INVALID_ARG = -1,   /* a NULL pointer, a bad size, overlapping channels */
    DSBT_ERR_UNSUPPORTED = -2,   /* N not a power of two in [16, 8192], l too large */
    DSBT_ERR_OOM = -3,           /* device or host allocation failed */
    DSBT_ERR_HIP = -4,           /* a HIP runtime call or kernel launch failed */
    DSBT_ERR_PLAN_MISMATCH = -5, /* call does not fit the plan (e.g. no potential set) */
    DSBT_ERR_NONFINITE = -6,     /* checked plan: a NaN or infinity in the data (dsbt_plan_opts.check_finite) */
    DSBT_ERR_NO_DEVICE = -7      /* no HIP device is visible */
};

typedef struct dsbt_plan_s* dsbt_plan;   /* opaque; owned by the library */

/* One radial channel.  N: grid size (power of two, 16..8192); ell: angular
 * momentum, 0 <= ell <= min(2N - 2, 255); rmax > 0: box radius (dr = rmax/N,
 * dk = pi/rmax); offset: first element of the channel in every data buffer,
 * counted in complex elements.  Channels must not overlap. */
typedef struct {
    int32_t N;
    int32_t ell;
    double rmax;
    int64_t offset;
} dsbt_channel;

/* data precision: complex64 data with FP32 arithmetic (FP32 tables from the
 * FP64 plan), complex128 data with FP64 arithmetic, or complex64 data with FP64
 * arithmetic and tables (rounded to FP32 only where data is stored; for long
 * propagations, where FP32 rounding of the constants biases the norm) */
enum { DSBT_C64 = 0, DSBT_C128 = 1, DSBT_C64_FP64 = 2 };
enum { DSBT_K_PLAIN = 0, DSBT_K_CORRECTED = 1 };     /* k_nl = n dk, or eq. kcorr roots */
enum { DSBT_SIGN_C = 0, DSBT_SIGN_PRINTED_F = 1 };   /* F with / without (-1)^ceil(l/2) */
enum { DSBT_MODE_BATCHED = 0, DSBT_MODE_PLAIN = 1 }; /* batched launches / one launch per channel and stage */
enum { DSBT_PLAN_ON_DEVICE = 0, DSBT_PLAN_ON_HOST = 1 };

typedef struct {
    int32_t precision;    /* DSBT_C64 (default), DSBT_C128 or DSBT_C64_FP64 */
    int32_t kinetic;      /* DSBT_K_PLAIN (default) or DSBT_K_CORRECTED: momenta of the kinetic
                             diagonal, see dsbt_kinetic_momenta */
    int32_t sign;         /* DSBT_SIGN_C (default): b_n ~ c_l(k_n) sqrt(w_n) */
    int32_t mode;         /* DSBT_MODE_BATCHED (default) or DSBT_MODE_PLAIN */
    int32_t plan_where;   /* DSBT_PLAN_ON_DEVICE (default): the FP64 DLOP recurrences and tile
                             blocks are computed by GPU kernels; DSBT_PLAN_ON_HOST: by host threads */
    int32_t tile;         /* moment tile B (power of two >= ceil((l+1)/2)); 0 = automatic */
    int32_t chans_per_block; /* channels per workgroup in the transform stage; 0 = automatic */
    int32_t algorithm;    /* DSBT_ALG_TILED (default) or DSBT_ALG_MONOMIAL, see below */
    int32_t check_finite; /* 0 (default) or 1: dsbt_forward, dsbt_inverse and dsbt_kinetic_step first
                             scan every channel of their input for NaN and infinities, synchronise
                             the stream and return DSBT_ERR_NONFINITE without touching the output if
                             one is found; dsbt_kinetic_step also scans psi after its steps and
                             returns DSBT_ERR_NONFINITE (psi then holds the result).  Checked calls
                             synchronise, so they cannot be captured in a graph. */
    int32_t reserved0;    /* 0 */
    /* Device allocator of the plan (both or neither; NULL: hipMalloc / hipFree).
     * Every device table, descriptor and plan-time scratch buffer of the plan is
     * obtained from dev_alloc(bytes, alloc_ctx) -- 256-byte aligned device memory
     * usable on any stream, or NULL on failure (then dsbt_plan_create returns
     * DSBT_ERR_OOM after handing back what it got) -- and handed back through
     * dev_free(ptr, alloc_ctx) by dsbt_plan_destroy or a failing create.  The
     * callbacks are called from the thread that makes the plan call, never from
     * a stream callback.  dsbt_plan_destroy does not synchronise: the caller
     * ensures no enqueued work still reads the plan (a caching allocator that
     * reuses freed blocks on other streams relies on that). */
    void* (*dev_alloc)(size_t bytes, void* alloc_ctx);
    void (*dev_free)(void* ptr, void* alloc_ctx);
    void* alloc_ctx;
    int32_t reserved[4];
} dsbt_plan_opts;

/* Moment-stage algorithm.  DSBT_ALG_TILED: the numerically stable tiled moment
 * form.  DSBT_ALG_MONOMIAL: the paper's own fast multiplication of Sec. 2.6
 * (eqs. DP_expan, fast_b_f, sum_in_b_f, rec_sum_b_f and, inverse, fast_f_b,
 * sum_in_f_b, fast_f_b_lowm, rec_sum_f_b): prefix and suffix sums of m^nu f_m
 * against the monomial coefficients xi_nu(n) of the DDLOP, in FP64, one wave per
 * channel.  Exact in exact arithmetic, but its sums cancel terms that grow
 * quickly with l, so its FP64 error rises from ~1e-15 at l <= 8 to ~1e-11 at
 * l = 16 and ~1e-7 at l = 24; it is kept to measure that.  Needs DSBT_C128 and
 * DSBT_MODE_BATCHED, l <= 128 and N^(l-1) within the FP64 range (else
 * DSBT_ERR_UNSUPPORTED).  Plan creation expands xi in binary128 on the host. */
enum { DSBT_ALG_TILED = 0, DSBT_ALG_MONOMIAL = 1 };

/* Fill *o with the defaults above (all zero). */
void dsbt_plan_opts_default(dsbt_plan_opts* o);

/* Build a plan for nch channels described by ch[0..nch).  The FP64 plan (DLOP
 * rows of T, the tiled moment tables, FFT twiddles) is generated once, cast to
 * the data precision and uploaded; `stream` orders the upload.  o may be NULL
 * (defaults).  On success *out receives the plan; on failure *out is NULL. */
dsbt_status dsbt_plan_create(dsbt_plan* out, const dsbt_channel* ch, int32_t nch,
                             const dsbt_plan_opts* o, void* stream);

/* Convenience: channels for every l in ells[0..nell) with a common N and rmax,
 * packed back to back in the order given; with all_m != 0 each l gets 2l+1
 * consecutive channels (m = -l..l). */
dsbt_status dsbt_plan_create_uniform(dsbt_plan* out, int32_t N, double rmax,
                                     const int32_t* ells, int32_t nell, int32_t all_m,
                                     const dsbt_plan_opts* o, void* stream);

dsbt_status dsbt_plan_destroy(dsbt_plan p);

/* Plan facts: number of channels, total complex elements a data buffer must
 * hold (max offset + N), data precision, and device bytes held by the plan. */
dsbt_status dsbt_plan_info(dsbt_plan p, int32_t* nch, int64_t* elems, int32_t* precision,
                           int64_t* table_bytes);

/* Forward transform b = T F psi for every channel (device pointers, layout as
 * above).  psi and b may be the same buffer.  Enqueued on `stream`. */
dsbt_status dsbt_forward(dsbt_plan p, const void* psi, void* b, void* stream);

/* Inverse transform psi = F^T T^T b for every channel.  b and psi may alias. */
dsbt_status dsbt_inverse(dsbt_plan p, const void* b, void* psi, void* stream);

/* Radial potential for the split step (Sec. 4.1).  V is a HOST array of FP64
 * values laid out like a data buffer (V[offset_c + i] = V_c(r_{i+1}), real);
 * dt is the time step tau.  The phase factors exp(-i s V tau/2) and
 * exp(-i K_n tau) are formed from FP64 angles reduced mod 2 pi.  Synchronises. */
dsbt_status dsbt_set_potential(dsbt_plan p, const double* V, double dt);

/* Imaginary-time method (Sec. 4.3, t -> -i t): the step factors become the
 * real decays exp(-V tau/2) and exp(-K_n tau), formed in FP64 and stored in
 * the plan's step tables (as complex values with zero imaginary part).
 * dsbt_kinetic_step then applies
 *     psi <- exp(-V tau/2) F^T T^T exp(-K tau) T F exp(-V tau/2) psi,
 * which damps every eigencomponent of energy E by exp(-E tau) per step (up to
 * the splitting error), so repeated steps followed by dsbt_orthonormalize
 * converge to the lowest bound states.  With this flag, dsbt_kinetic_step
 * takes no strengths (s must be NULL) and dsbt_step_grad_s returns
 * DSBT_ERR_PLAN_MISMATCH until the potential is set again without it. */
enum { DSBT_TIME_IMAGINARY = 1 };

/* dsbt_set_potential with flags: 0 (real time, the same as dsbt_set_potential)
 * or DSBT_TIME_IMAGINARY.  Other bits: DSBT_ERR_INVALID_ARG.  Synchronises. */
dsbt_status dsbt_set_potential_ex(dsbt_plan p, const double* V, double dt, int32_t flags);

enum {
    DSBT_STEP_ADJOINT = 1,   /* apply U^H (conjugated phases), steps in reverse order */
    DSBT_STEP_GRAPH = 2,     /* capture the nsteps launches once in a hipGraph and replay it; the
                                strengths are first copied (on `stream`) into a plan buffer the graph
                                reads, so only a new psi, nsteps or flags value captures again */
    DSBT_STEP_RESIDENT = 4   /* one launch that keeps each channel in LDS for all steps */
};

/* nsteps split-operator steps in place on psi (device).  s: device FP32 array
 * of nsteps potential strengths (step t uses s[t]; NULL means all ones); with
 * DSBT_STEP_ADJOINT the steps run t = nsteps-1 .. 0.  Needs dsbt_set_potential. */
dsbt_status dsbt_kinetic_step(dsbt_plan p, void* psi, int32_t nsteps, const float* s,
                              int32_t flags, void* stream);

/* Gradient of a real loss L with respect to the strength s_t of one step,
 * given psi_t, psi_{t+1} = U_t psi_t and the adjoint states lam_t = U_t^H lam_{t+1},
 * lam_{t+1} (PyTorch convention: lam = 2 dL/d conj(psi)):
 *   out[0] = (tau/2) sum_i V_i Im(conj(lam_{t+1,i}) psi_{t+1,i} + conj(lam_{t,i}) psi_{t,i}).
 * out is a device FP64 scalar; written, not accumulated. */
dsbt_status dsbt_step_grad_s(dsbt_plan p, const void* psi_t, const void* psi_t1,
                             const void* lam_t, const void* lam_t1, double* out, void* stream);

/* Backward pass of one checkpoint segment of the adjoint method (Sec. 4.1:
 * U_t^H = U_t^-1, so lam_t = U_t^H lam_{t+1} is a split step with conjugated
 * phases).  Inputs: psi_a, the state before step a; s, the n strengths
 * s_a .. s_{a+n-1} (device FP32); lam = lam_{a+n} (device, data layout).
 * The call recomputes psi_{a+1} .. psi_{a+n} from psi_a, then for
 * t = a+n-1 .. a forms lam_t and gs[t-a] = dL/ds_t exactly as
 * dsbt_step_grad_s does, and leaves lam_a in lam (psi_a is not written).
 * gs: device FP64 array of n values, written.  All work runs on plan-owned
 * buffers (2n + 4 states and n x nch doubles, grown through the plan's
 * allocator to the largest n seen; a call that grows them synchronises
 * `stream`): the inputs are copied in and the results out on `stream`.
 * Batched plans run the recompute and the adjoint steps side by side on
 * `stream` and a second stream of the plan, joined before the gradients.
 * flags: 0, or DSBT_STEP_GRAPH: the segment's launches (n steps, n adjoint
 * steps, the gradient reductions) are captured
 * once in a hipGraph on those buffers and replayed, so every later call with
 * the same n replays it.  Checked plans scan psi_a and lam before and lam
 * after, synchronising, and do not use the graph.  Needs dsbt_set_potential
 * in real time (else DSBT_ERR_PLAN_MISMATCH); n < 1 or other flag bits:
 * DSBT_ERR_INVALID_ARG. */
dsbt_status dsbt_adjoint_segment(dsbt_plan p, const void* psi_a, int32_t nsteps, const float* s, void* lam,
                                 double* gs, int32_t flags, void* stream);

/* dsbt_step_grad_s for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and result, with the per-channel FP64 partial sums in a
 * fixed device array of DSBT_NOALLOC_MAX_CHANNELS doubles (512 KiB) that the
 * library holds on each GPU it runs on until the process ends, instead of the
 * plan's buffer.  The call itself allocates nothing (its first call on a
 * device only looks up that array's address).  Every call on one GPU shares
 * the array: calls that overlap on a GPU (several streams or host threads)
 * race and must be serialised by the caller.  A plan with more than
 * DSBT_NOALLOC_MAX_CHANNELS channels: DSBT_ERR_UNSUPPORTED.  Other errors as
 * dsbt_step_grad_s. */
#define DSBT_NOALLOC_MAX_CHANNELS 65536
dsbt_status dsbt_step_grad_s_noalloc(dsbt_plan p, const void* psi_t, const void* psi_t1,
                                     const void* lam_t, const void* lam_t1, double* out, void* stream);

/* Energy terms of eq. H_DVR per channel (Sec. 4.1, used for the bound-state
 * energies of Sec. 4.3): with b = T F psi,
 *     out[3c + 0] = sum_i |psi_i|^2,
 *     out[3c + 1] = sum_i V_i |psi_i|^2,
 *     out[3c + 2] = sum_n K_n |b_n|^2,   K_n = k_n^2/2 as in dsbt_kinetic_momenta,
 * so the energy of channel c is (out[3c+1] + out[3c+2]) / out[3c+0].  V is the
 * potential of the last dsbt_set_potential(_ex) (DSBT_ERR_PLAN_MISMATCH if none).
 * psi: device data buffer; work: device data buffer of the plan's size that
 * receives b (must not alias psi); out: device FP64 array of 3 * nch values,
 * written (not accumulated) in FP64 sums.  Enqueued on `stream`. */
dsbt_status dsbt_energy(dsbt_plan p, const void* psi, void* work, double* out, void* stream);

/* Gram-Schmidt orthonormalisation within sets of channels, in place on the
 * device buffer psi (the orthogonalisation to lower states of Sec. 4.3).  sets
 * is a HOST array of nsets + 1 channel indices, strictly increasing within
 * [0, nch]; set k is the channels sets[k] .. sets[k+1]-1, which must share N
 * (else DSBT_ERR_INVALID_ARG).  In channel order, each channel of a set loses
 * its components <psi_i|psi_j> psi_i along the already orthonormalised
 * channels i of its set (one at a time, FP64 sums), then is scaled to unit
 * norm; a channel whose norm is zero is left zero.  Channels outside every set
 * are not touched.  The set table is kept in the plan: a call with a table that
 * differs from the previous call's synchronises `stream` and uploads it, other
 * calls only enqueue one launch on `stream`. */
dsbt_status dsbt_orthonormalize(dsbt_plan p, void* psi, const int32_t* sets, int32_t nsets, void* stream);

/* Autotuner: picks the moment tile B and the channels per moment work item for
 * a channel set by measurement.  Candidates: tile 0 (the plan's own choice
 * per l), 32 and 64, crossed with chans_per_block 0 (the plan's own choice),
 * 8 and 4; candidates the channels do not admit are skipped.  Each is built
 * as a plan from *base (NULL = defaults) and timed with HIP events over nrep
 * forward + inverse pairs (after one untimed pair) on device scratch buffers
 * that the call allocates and frees.  *best receives *base with the fastest
 * tile and chans_per_block; ms (may be NULL) the time of one pair in ms.
 * cache_path (may be NULL): a JSON-lines file; a line whose key matches this
 * device architecture, precision, mode, algorithm and (N, l, rmax) multiset is
 * returned without timing, and a new result is appended.  Synchronises
 * `stream`.  DSBT_ERR_UNSUPPORTED if no candidate is admitted (the message
 * is the last candidate's), DSBT_ERR_NO_DEVICE without a device. */
dsbt_status dsbt_autotune(const dsbt_channel* ch, int32_t nch, const dsbt_plan_opts* base, int32_t nrep,
                          const char* cache_path, dsbt_plan_opts* best, double* ms, void* stream);

/* Angular transform Y = P Phi of the DSBT-DVR solver (Sec. 4.1), applied at
 * every radial point: grid values on N_theta Gauss-Legendre nodes eta_j
 * (ascending) and N_phi = 2M + 1 azimuths phi_k = 2 pi k / N_phi, carrying the
 * weights sqrt(w_j dphi), map to coefficients of the spherical harmonics
 * (l, m), m = -M..M, l = |m| .. |m| + N_theta - 1.  Phi is the unitary DFT
 * exp(-i m phi_k) / sqrt(N_phi) (the projection onto Y_lm); P, per m, holds
 * the associated Legendre functions Pbar_l^m(eta_j) sqrt(w_j) (unit norm on
 * [-1, 1], Condon-Shortley phase) orthonormalised on the quadrature in l order
 * (built as sqrt(w_j (1 - eta_j^2)^|m|) times the orthonormal polynomials of
 * those weights, by a Lanczos recurrence), so Y is unitary.  Layouts (complex, interleaved, radius fastest):
 *   grid  psi[j][k][i]   (j < N_theta, k < N_phi, i < Nr)
 *   coef  c[q][t][i]     (m = q - M, l = |m| + t): channel q N_theta + t of a
 *                        DSBT plan with N = Nr, that l and offset (q N_theta + t) Nr.
 * 1 <= N_theta <= 64, N_phi odd in [1, 63] (else DSBT_ERR_UNSUPPORTED). */
typedef struct dsbt_sht_s* dsbt_sht;   /* opaque; owns its tables and an Nr N_theta N_phi workspace */

/* Host: nodes eta[N_theta], weights w[N_theta], azimuths phi[N_phi] (any may be NULL). */
dsbt_status dsbt_sht_grid(int32_t n_theta, int32_t n_phi, double* eta, double* w, double* phi);
/* Host FP64 P blocks for testing, P[(q N_theta + t) N_theta + j]. */
dsbt_status dsbt_sht_host_tables(int32_t n_theta, int32_t n_phi, double* P);
/* precision: DSBT_C64 (complex64 data, FP32 tables and arithmetic) or
 * DSBT_C128 (complex128, FP64).  Allocates its tables and workspace. */
dsbt_status dsbt_sht_create(dsbt_sht* out, int32_t Nr, int32_t n_theta, int32_t n_phi, int32_t precision);
dsbt_status dsbt_sht_destroy(dsbt_sht s);
/* coef = Y grid and grid = Y^H coef on device buffers of Nr N_theta N_phi
 * complex values; enqueued on `stream` (two launches through the workspace,
 * so calls on one transform must not overlap); grid and coef may alias. */
dsbt_status dsbt_sht_forward(dsbt_sht s, const void* grid, void* coef, void* stream);
dsbt_status dsbt_sht_inverse(dsbt_sht s, const void* coef, void* grid, void* stream);
/* Potential factor of the 3D split step (Sec. 4.1, coordinate gauge), in place
 * on a grid buffer: grid *= exp(-i (V0 + F V1) dt/2), V0 and V1 device FP64
 * arrays in grid layout (either may be NULL: zero), F the step's field strength;
 * angles formed and reduced mod 2 pi in FP64.  With Y and a plan over
 * Y's channels whose potential is zero, one step is: this call, Y forward,
 * dsbt_kinetic_step (B^T exp(-i K dt) B), Y inverse, this call. */
dsbt_status dsbt_sht_potential_phase(dsbt_sht s, void* grid, const double* V0, const double* V1, double F, double dt,
                                     void* stream);
/* Velocity gauge (Sec. 4.1): coefficient channels in slot order (c[q][t][i],
 * i the DSBT slot) to the unified momentum grid k~_n = n dk, n = 1..Nr
 * (eq. tilde_k_grid) and back.  Forward (inverse = 0): dst = i^-l src, with
 * the n = 0 slot of odd l moved to n = Nr; then dsbt_sht_inverse gives
 * Ytilde^H c, the plane-wave grid [j][k][n].  Inverse (inverse != 0) undoes
 * it (i^l).  src and dst must not overlap (DSBT_ERR_INVALID_ARG). */
dsbt_status dsbt_sht_momentum_order(dsbt_sht s, const void* src, void* dst, int32_t inverse, void* stream);

/* Diagonal tables of the 3D split step, FP64, computed on the host and copied
 * to the caller's device array (synchronises `stream`):
 *   dsbt_sht_kinetic:     K[c Nr + i] = k_i^2 / 2 for coefficient channel c = q N_theta + t
 *                         (l = |q - M| + t) and slot i, the kinetic diagonal of eq. KinMat with
 *                         the momenta of dsbt_kinetic_momenta(Nr, l, rmax, kinetic);
 *   dsbt_sht_momentum_pz: Pz[(j N_phi + k) Nr + n - 1] = -2 k~_n eta_j, n = 1..Nr, on the
 *                         unified momentum grid k~_n = n pi / rmax (eq. tilde_k_grid), so that
 *                         dsbt_sht_potential_phase(V1 = Pz, F = A) multiplies by
 *                         exp(i A k~_n eta_j dt), the A.P factor of eq. H_DVR for A along z.
 * Both arrays hold Nr N_theta N_phi doubles; rmax > 0 (else DSBT_ERR_INVALID_ARG). */
dsbt_status dsbt_sht_kinetic(dsbt_sht y, double rmax, int32_t kinetic, double* K, void* stream);
dsbt_status dsbt_sht_momentum_pz(dsbt_sht y, double rmax, double* Pz, void* stream);

/* One 3D split step (Sec. 4.1) in place on a grid buffer, enqueued on `stream`.
 * p: a plan over the transform's channels (channel q N_theta + t: N = Nr, l = |m| + t,
 * offset (q N_theta + t) Nr) with the potential set to zero for this dt; work (and
 * work1, work2): device buffers of the grid size, not aliasing grid.
 * Coordinate gauge: grid <- exp(-i U dt/2) Y^H B^T exp(-i K dt) B Y exp(-i U dt/2) grid,
 * U = V0 + F V1 (device FP64 grid arrays, either may be NULL).
 * Velocity gauge (A along z): the printed sequence through the momentum grid,
 * with K the kinetic energies per channel slot (device FP64, coefficient
 * layout, from dsbt_sht_kinetic) and Pz = -2 k~_n eta_j on the momentum grid
 * (device FP64, from dsbt_sht_momentum_pz), so that the A.P factor is
 * exp(i A k~_n eta_j dt).  The first failing call's status
 * is returned (later calls are not enqueued). */
dsbt_status dsbt_step3d(dsbt_sht y, dsbt_plan p, void* grid, void* work, const double* V0, const double* V1, double F,
                        double dt, void* stream);
dsbt_status dsbt_step3d_velocity(dsbt_sht y, dsbt_plan p, void* grid, void* work1, void* work2, const double* V0,
                                 const double* K, const double* Pz, double A, double dt, void* stream);

/* Stage timing.  With profiling enabled, every stage launch made by
 * dsbt_forward, dsbt_inverse and dsbt_kinetic_step (outside graph capture) is
 * bracketed by HIP events recorded on the launch stream.  enable == 1 clears
 * the accumulators and starts recording; enable == 2 resumes recording and
 * keeps them (to sample some launches of a longer run); enable == 0 stops
 * recording.  Adds two event records per recorded launch. */
dsbt_status dsbt_profile_enable(dsbt_plan p, int32_t enable);
enum { DSBT_STAGE_SINCOS = 0, DSBT_STAGE_MOMENT = 1, DSBT_NUM_STAGES = 2 };
/* Synchronises on the recorded events and returns, per stage (index as above,
 * nstages <= DSBT_NUM_STAGES), the summed milliseconds and the launch count. */
dsbt_status dsbt_profile_read(dsbt_plan p, double* ms, int64_t* launches, int32_t nstages);

/* Host FP64 moment tables of one (N, l, B) for testing the plan without a GPU.
 * Writes R*R*NT doubles, R = B + ceil(l/2), NT = N/B: block J (row-major,
 * M[r][q]) maps [g_J ; mu_J] to [b_J ; mu_{J+1}] for the tile of slots
 * [J B, J B + B).  If out is NULL or out_len is too small only *needed is set. */
dsbt_status dsbt_host_ftb_tables(int32_t N, int32_t ell, int32_t B, double* out,
                                 int64_t out_len, int64_t* needed);

/* Host FP64 tables of the monomial variant (DSBT_ALG_MONOMIAL) for one (N, l),
 * for testing without a GPU.  With k = ceil(l/2), p = 1 for even l (else 0),
 * n_0 = ceil((l+1)/2) and R = N + p - n_0 regular rows n = n_0 .. N + p - 1:
 * xi[(n - n_0) k + q] = xi_nu(n) of eq. DP_expan for nu = (l+1) mod 2 + 2q,
 * alpha[n - n_0] = alpha_n (Sec. 2.4), comp[q N + j] = T_{p+q, j+p} (the
 * completion rows, slot order).  sizes (3 values, may be NULL) receives
 * R k, R and k N; any array may be NULL (not written), else it must hold its
 * size. */
dsbt_status dsbt_host_monomial_tables(int32_t N, int32_t ell, double* xi, double* alpha, double* comp,
                                      int64_t* sizes);

/* The same blocks computed by the device plan generator (the FP64 kernels that
 * dsbt_plan_create runs with DSBT_PLAN_ON_DEVICE) on the current HIP device,
 * l <= 255; `stream` orders the work and is synchronised before return.  The
 * generator allocates its scratch (about (N^2/2 + ceil(l/2) N^2/(2B)) doubles)
 * for the call and frees it.  Returns DSBT_ERR_NO_DEVICE without a device. */
dsbt_status dsbt_device_ftb_tables(int32_t N, int32_t ell, int32_t B, double* out,
                                   int64_t out_len, int64_t* needed, void* stream);

/* The momenta k_n of the kinetic diagonal K_n = k_n^2/2 that dsbt_set_potential
 * uses for a channel (N, ell, rmax), in slot order (N doubles written to k):
 * the completion rows n < n_0 take N dk (their energy is the top of the grid);
 * regular rows take n dk (DSBT_K_PLAIN, eq. tilde_k_grid) or x_j / rmax
 * (DSBT_K_CORRECTED, eq. kcorr), x_j the j-th positive root, j = n - n_0 + 1,
 * of chi_l(x) = x j_l(x) for even l and of chi_l'(x) for odd l (Sec. 3).
 * Host computation in FP64. */
dsbt_status dsbt_kinetic_momenta(int32_t N, int32_t ell, double rmax, int32_t kinetic, double* k);

const char* dsbt_status_string(dsbt_status s);
const char* dsbt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DSBT_H */
