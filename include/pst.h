/*
 * pst.h -- C ABI of the MI355X-native pseudospectral turbulence hot path.
 *
 * The library evaluates and time-steps the incompressible Navier-Stokes
 * equations (the paper's eq. mom + eq. divv with theta = 0) and, as further
 * solvers, incompressible MHD (eq. uMHD, eq. bMHD) and the Boussinesq
 * equations of a stably stratified fluid (eq. mom, eq. temp, eq. divv: the
 * velocity and the temperature fluctuation theta, coupled by the buoyancy
 * terms -N theta zhat and +N w of Brunt-Vaisala frequency N) on a periodic n^3 grid of
 * [0, 2 pi)^3 with the Fourier-Galerkin pseudospectral method of Sec. 2:
 * nonlinear terms are formed in physical space between backward and forward
 * 3D transforms, pressure is applied by projecting onto divergence-free
 * fields, and an explicit Runge-Kutta scheme advances the Fourier
 * coefficients.  Every step runs in hand-written HIP kernels for gfx950.
 *
 * Plans follow the create / execute / destroy life cycle of the paper's
 * transform plans (Sec. 3.2): a plan owns every device buffer it allocates
 * and borrows the caller's HIP stream.  All functions return a pst_status;
 * 0 (PST_OK) is success, as for the runtime return codes the paper binds
 * (Sec. 3.1).  Nothing throws or aborts across this interface.  Errors are
 * sticky per plan: pst_last_error() returns the message of the last failure.
 * Plans are not thread-safe; use one plan per host thread.
 *
 * Conventions
 *  - Transform (eq. fftsum): forward sign -, scaled by 1/n^3 so that
 *    u(x) = sum_k uhat(k) exp(i k.x); backward sign +, unscaled.
 *  - Physical layout:  real    [ncomp][n][n][n]       (z, y, x; x fastest).
 *  - Spectral layout:  complex [ncomp][n][n][n/2+1]   (kz, ky, kx; kx fastest),
 *    interleaved (re, im).  Index p on a full axis is wavenumber p for p < n/2,
 *    p - n otherwise; kx runs over 0..n/2 (Hermitian half, Sec. 2).
 *  - Element type follows the plan precision: float (PST_FP32) or double
 *    (PST_FP64).  Diagnostics are always double.
 *  - Dealiasing: cube truncation max(|kx|,|ky|,|kz|) <= K, K = ceil(n/3) - 1
 *    (the largest K with 3K < n, alias-free for quadratic products).  The
 *    state only ever holds these modes.
 *  - Time stepping: Lawson integrating factor E = exp(-nu |k|^2 h / 2)
 *    (eta for b, kappa = eta for theta) with Heun RK2 or classical RK4; the
 *    buoyancy coupling is part of the explicit right-hand side.
 *  - "device" pointers are HIP device allocations on the current device;
 *    "host" pointers are ordinary host memory.
 *  - Stream-ordered calls only enqueue work on the plan's stream; synchronous
 *    calls wait for it.
 */
#ifndef PST_H
#define PST_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PST_OK = 0,
    PST_ERR_INVALID_ARG = 1,   /* bad pointer, size, enum or state */
    PST_ERR_UNSUPPORTED_N = 2, /* n not in the supported set */
    PST_ERR_OOM = 3,           /* device allocation failed */
    PST_ERR_HIP = 4,           /* a HIP runtime call failed */
    PST_ERR_NONFINITE = 5,     /* a diagnostic found NaN or Inf */
    PST_ERR_UNSUPPORTED = 6    /* option not implemented for this plan */
} pst_status;

/* GPE: the Gross-Pitaevskii equation of a complex wavefunction psi (eq. gpe),
 *   d psi / dt = i alpha Lap psi - i beta |psi|^2 psi,
 * on the whole spectrum (c2c transforms), its cubic product dealiased by the
 * cube |k_i| <= K = ceil(n/4) - 1 (4K < n), the linear part taken exactly by
 * the unitary integrating factor exp(-i alpha |k|^2 h / 2). */
typedef enum { PST_NS = 0, PST_MHD = 1, PST_BOUSSINESQ = 2, PST_GPE = 3 } pst_solver;
typedef enum { PST_FP32 = 0, PST_FP64 = 1 } pst_precision;
/* Dealiasing of the nonlinear terms (2/3 rule, K = ceil(n/3) - 1):
 * CUBE keeps max(|kx|, |ky|, |kz|) <= K; SPHERE keeps |k|^2 <= K^2.  The state
 * always holds the cube; under SPHERE the modes between sphere and cube get
 * no nonlinear term (they evolve by the linear part alone).  NONE (tests
 * only: it shows the aliasing the other two remove) uses K = n/2 - 1, i.e.
 * keeps every mode except the Nyquist ones, so products alias.  Ensembles use
 * the cube. */
typedef enum { PST_DEALIAS_CUBE = 0, PST_DEALIAS_SPHERE = 1, PST_DEALIAS_NONE = 2 } pst_dealias;
/* U: velocity (3 components); B: magnetic field (MHD, 3 components); THETA:
 * temperature fluctuation (Boussinesq, 1 component: physical [1][n][n][n],
 * spectral [1][n][n][n/2+1]); PSI: the wavefunction (GPE, 1 complex
 * component: physical complex [1][n][n][n], spectral complex [1][n][n][n], kx
 * on the full axis like ky and kz). */
typedef enum { PST_FIELD_U = 0, PST_FIELD_B = 1, PST_FIELD_THETA = 2, PST_FIELD_PSI = 3 } pst_field;
typedef enum { PST_SPACE_PHYS = 0, PST_SPACE_SPEC = 1 } pst_space;
typedef enum { PST_MEM_HOST = 0, PST_MEM_DEVICE = 1 } pst_mem;

enum {
    PST_FLAG_LINEAR_ONLY = 1u, /* nonlinear operator replaced by 0 (tests of the integrating factor) */
    PST_FLAG_TIMERS = 2u       /* record HIP events around every kernel (see pst_timer_read) */
};

typedef struct {
    int n;            /* grid points per direction; see pst_supported_n() */
    int solver;       /* pst_solver */
    int precision;    /* pst_precision */
    int rk_order;     /* 2 (Heun) or 4 (classical) */
    double nu;        /* kinematic viscosity */
    double eta;       /* magnetic diffusivity (MHD) or scalar diffusivity kappa (Boussinesq) */
    double dt;        /* time step h */
    int dealias;      /* pst_dealias */
    unsigned flags;   /* PST_FLAG_* */
    double nbv;       /* Brunt-Vaisala frequency N (Boussinesq; ignored otherwise) */
    double alpha;     /* GPE: coefficient of the Laplacian (hbar / 2m); ignored otherwise */
    double beta;      /* GPE: coupling of |psi|^2 psi (g / hbar); ignored otherwise */
    /* Anisotropic grids (Sec. 2: the point counts N_i and box lengths L_i may
     * differ per direction): points per direction (each a supported n; 0
     * selects n) and box lengths (0 selects 2 pi).  Physical wavenumbers are
     * 2 pi p / L_i, every axis has its own cutoff K_i, and layouts become
     * physical [c][nz][ny][nx], spectral [c][nz][ny][nx/2+1] (GPE [c][nz][ny][nx]).
     * SPHERE needs a cubic 2 pi grid; ensembles and the neural operator are cubic. */
    int nx, ny, nz;
    double lx, ly, lz;
} pst_params;

typedef struct {
    int n, kcut;              /* grid size and dealias cutoff K */
    int ncomp;                /* state components: 3 (NS), 6 (MHD: u, b), 4 (Boussinesq: u, theta), 1 (GPE) */
    size_t modes_per_comp;    /* stored modes per component: (K+1)(2K+1)^2, GPE (2K+1)^3 */
    size_t workspace_bytes;   /* device bytes owned by the plan */
    int radices[4];           /* FFT radix schedule of the n-point transforms (0-terminated) */
    int tile_lines;           /* lines per workgroup in the strided passes */
    long long steps_done;     /* time steps taken since the last set_state */
    int nx, ny, nz;           /* points per direction (n = nz) */
    int kcut_x, kcut_y;       /* dealias cutoffs of x and y (kcut: z) */
    int nshells;              /* shells a pst_spectrum call needs at least */
} pst_info;

/* Kernel kinds reported by pst_timer_read (PST_FLAG_TIMERS). */
typedef enum {
    PST_K_ZINV = 0,   /* backward z transform + spectral curl */
    PST_K_YINV = 1,   /* backward y transform */
    PST_K_XPASS = 2,  /* fused backward x (c2r), cross products, forward x (r2c) */
    PST_K_YFWD = 3,   /* forward y transform */
    PST_K_ZFWD = 4,   /* forward z transform + projection + forcing + RK update */
    PST_K_FFTX = 5,   /* standalone transforms: x (r2c / c2r) */
    PST_K_FFTY = 6,   /* standalone transforms: y */
    PST_K_FFTZ = 7,   /* standalone transforms: z */
    PST_K_OTHER = 8,  /* gathers, scatters, reductions */
    PST_K_COUNT = 9
} pst_kernel_kind;

typedef struct pst_plan pst_plan;

/* Text of a status code (static storage). */
const char *pst_status_str(pst_status s);

/* Message of the last failure on this plan ("" if none; plan may be NULL for
 * failures of pst_plan_create, which are kept per host thread). */
const char *pst_last_error(const pst_plan *plan);

/* 1 if n is supported by this build, else 0.  Supported n are products of 2
 * and 3 with a compiled FFT schedule: 16, 24, 32, 48, 64, 96, 128, 256, 512,
 * 1024. */
int pst_supported_n(int n);

/* Create a plan (Sec. 3.2, plan creation): validates p, allocates the state,
 * the pass buffers, and the twiddle and integrating-factor tables, generated
 * in FP64 or better and rounded once to the plan precision (FP32 transforms
 * evaluate their twiddles with the hardware sine and cosine instead of
 * reading the table).  hip_stream (hipStream_t, may be NULL
 * for the null stream) is borrowed and must outlive the plan.  The state
 * starts at zero.  Errors: INVALID_ARG, UNSUPPORTED_N, UNSUPPORTED, OOM, HIP. */
pst_status pst_plan_create(const pst_params *p, void *hip_stream, pst_plan **out);

/* Free everything the plan owns (synchronises its stream).  NULL is a no-op. */
void pst_plan_destroy(pst_plan *plan);

/* Load field u (b for MHD, theta for Boussinesq) from src.  PHYS: real
 * [nc][n][n][n]; SPEC: complex [nc][n][n][n/2+1], nc = 3 (u, b) or 1 (theta).
 * INVALID_ARG for a field the solver does not have.  The data is copied: modes outside the dealiasing cube
 * are dropped and the kx = 0 plane is made Hermitian ((X(k) + conj X(-k))/2).
 * mem says where src lives; a HOST copy is synchronous, a DEVICE copy is
 * stream-ordered.  Resets the step counter. */
pst_status pst_set_state(pst_plan *plan, int field, int space, const void *src, int mem);

/* Write field u (b, theta) to dst in the layout of pst_set_state (all modes
 * outside the cube are zero).  HOST: synchronous; DEVICE: stream-ordered. */
pst_status pst_get_state(pst_plan *plan, int field, int space, void *dst, int mem);

/* Constant forcing fhat added to the projected nonlinear term of u, spectral
 * layout [3][n][n][n/2+1]; it should be solenoidal (it is dealiased, not
 * projected).  NULL removes the forcing.  Navier-Stokes and Boussinesq only.
 * Synchronous for HOST. */
pst_status pst_set_forcing(pst_plan *plan, const void *fhat, int mem);

/* Nonlinear right-hand side of the state in state_dev (device, spectral
 * layout; NS: [3] comps of u, MHD: [6] = u then b, Boussinesq: [4] = u then
 * theta, GPE: [1] psi on the full spectrum), written to rhs_dev (same layout);
 * GPE: N = -i beta D F[|psi|^2 psi];  NS  N = D P F[u x w] + f;  MHD
 * N_u = D P F[u x w + j x b], N_b = D (i k x F[u x b]);  Boussinesq
 * N_u = D P (F[u x w] - N thetahat zhat) + f, N_theta = D (-F[u . grad theta]
 * + N w_z) (eq. mom, eq. temp; u . grad u in rotational form, its gradient
 * part absorbed by the projection).  Viscous and diffusive terms are
 * excluded.  Stream-ordered.  Does not touch the plan's state. */
pst_status pst_rhs(pst_plan *plan, const void *state_dev, void *rhs_dev);

/* Advance the plan's state by nsteps integrating-factor RK steps.
 * Stream-ordered. */
pst_status pst_step(pst_plan *plan, int nsteps);

/* Energies E = 1/2 <|v|^2> = 1/2 sum_k w |vhat|^2 (w = 1 on kx = 0, else 2)
 * of u and of b (MHD) or theta (Boussinesq: 1/2 <theta^2>); out[1] = 0 for
 * NS.  GPE: out[0] = particle number sum_k |psihat|^2 = <|psi|^2>, out[1] =
 * kinetic energy alpha sum_k |k|^2 |psihat|^2 (the interaction energy
 * beta/2 <|psi|^4> needs psi at the grid points: pst_get_state PHYS).
 * Accumulated in double.  Synchronous.  NONFINITE if either is NaN/Inf. */
pst_status pst_energy(pst_plan *plan, double out[2]);

/* Enstrophies Z = 1/2 sum_k w |k|^2 |vhat|^2 of u and of b or theta (out[1]
 * = 0 for NS; for a solenoidal field Z = 1/2 <|curl v|^2>, for theta
 * 1/2 <|grad theta|^2>), accumulated in double; with the energies they give
 * the dissipation rate -2 (nu Z_u + eta Z_2) of the unforced equations.
 * Synchronous.  NONFINITE if either is NaN/Inf. */
pst_status pst_enstrophy(pst_plan *plan, double out[2]);

/* Dealias and project ngroups vector fields given in the spectral layout
 * ([ngroups][3][nz][ny][nx/2+1], device, the plan's precision), in place: modes
 * outside the dealiasing cube are zeroed, the others projected onto
 * divergence-free fields (Sec. 2: pressure by projection; the k = 0 mode is
 * kept).  energy / enstrophy (host double[ngroups], either may be NULL) receive
 * 1/2 sum w |v|^2 and 1/2 sum w |k|^2 |v|^2 of each projected group; the call
 * is then synchronous, else stream-ordered.  UNSUPPORTED for GPE plans. */
pst_status pst_project(pst_plan *plan, void *spec_dev, int ngroups, double *energy, double *enstrophy);

/* Shell spectrum E(s) = 1/2 sum_{floor(|k|+1/2) = s} w |vhat|^2 for
 * s = 0..nshells-1 (double; GPE: the number spectrum sum_shell |psihat|^2),
 * summed in a fixed order (bitwise repeatable).
 * nshells must be in [floor(sqrt(3) K + 1/2) + 1, 2048].  Synchronous. */
pst_status pst_spectrum(pst_plan *plan, int field, double *Ek, int nshells);

/* Standalone unpruned 3D transforms of nfields fields (device pointers, the
 * plan's n and precision).  r2c: real [nfields][n][n][n] -> complex
 * [nfields][n][n][n/2+1], scaled by 1/n^3.  c2r: the inverse, unscaled,
 * imaginary parts of the self-conjugate points ignored; in is not modified.
 * in and out must not overlap.  Stream-ordered; c2r uses plan workspace. */
pst_status pst_fft_r2c(pst_plan *plan, const void *in, void *out, int nfields);
pst_status pst_fft_c2r(pst_plan *plan, const void *in, void *out, int nfields);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * transform of pst_fft_c2r without a plan and without any allocation.  in:
 * complex [nfields][n][n][n/2+1], out: real [nfields][n][n][n] (device, the
 * element type of precision), on hip_stream (may be NULL).  The n roots of
 * unity (regenerated every call in FP64, rounded once) and the pass workspace
 * live in a static device array of PST_NOALLOC_SCRATCH_BYTES per GPU, held
 * until the process ends; pst_fft_c2r_noalloc_bytes(n, precision, nfields)
 * gives what a call needs (0 for invalid arguments) and calls needing more
 * than the limit fail with INVALID_ARG (e.g. n = 128 takes up to 3 FP64 or 7
 * FP32 fields, n = 256 is refused).  Nothing in the array needs to start at
 * zero.  Every call on one GPU shares that GPU's array: calls that overlap on
 * one GPU (other streams, other host threads) race and must be serialised by
 * the caller.  Stream-ordered; errors are reported through pst_last_error(NULL). */
#define PST_NOALLOC_SCRATCH_BYTES (64u << 20)
size_t pst_fft_c2r_noalloc_bytes(int n, int precision, int nfields);
pst_status pst_fft_c2r_noalloc(int n, int precision, const void *in, void *out, int nfields, void *hip_stream);

/* Sizes and schedule of the plan. */
pst_status pst_query(const pst_plan *plan, pst_info *info);

/* With PST_FLAG_TIMERS: synchronise, and return per kernel kind the summed
 * duration in ms and the launch count since the last reset (arrays of
 * PST_K_COUNT entries; either may be NULL), then reset if reset != 0.
 * Durations come from HIP events recorded on the plan's stream around each
 * launch.  Without the flag: UNSUPPORTED. */
pst_status pst_timer_read(pst_plan *plan, double *ms, long long *count, int reset);

/* ------------------------------------------------------------------------
 * Ensembles: many independent Navier-Stokes runs of uneven n advanced
 * together.  This batches what the paper batches over CUDA streams (Sec. 3.3:
 * many small transforms in flight at once) but keeps every run resident on
 * the device and advances all of them with one persistent kernel launch per
 * time step (device-wide barriers between the transform passes), replayed
 * from a captured HIP graph.
 * ---------------------------------------------------------------------- */
typedef struct pst_ensemble pst_ensemble;

enum {
    PST_ENS_PERSISTENT_GRAPH = 0, /* persistent step kernel replayed from a HIP graph (default) */
    PST_ENS_PERSISTENT = 1,       /* persistent step kernel, launched directly */
    PST_ENS_BATCHED = 2,          /* one launch per (pass, grid size) covering all runs of that size */
    PST_ENS_SEQUENTIAL = 3,       /* one launch per (pass, run) */
    PST_ENS_BATCHED_GRAPH = 4     /* the batched launches of one step replayed from a HIP graph */
};

/* Create nruns runs; run r has grid n[r] (each of 32, 48, 64, 96; at most 4
 * distinct sizes) and the parameters in common (solver NS, precision FP32,
 * rk_order 2 or 4, nu, dt; flags 0).  States start at zero.  hip_stream is
 * borrowed.  Errors: INVALID_ARG, UNSUPPORTED_N, UNSUPPORTED, OOM, HIP. */
pst_status pst_ensemble_create(int nruns, const int *n, const pst_params *common, void *hip_stream,
                               pst_ensemble **out);
void pst_ensemble_destroy(pst_ensemble *ens);
const char *pst_ensemble_last_error(const pst_ensemble *ens);

/* State of run `run`: complex float [3][n][n][n/2+1] spectral layout of
 * pst_set_state (dealiased, kx = 0 plane made Hermitian).  HOST copies are
 * synchronous, DEVICE copies stream-ordered. */
pst_status pst_ensemble_set_state(pst_ensemble *ens, int run, const void *uhat, int mem);
pst_status pst_ensemble_get_state(pst_ensemble *ens, int run, void *uhat, int mem);

/* Advance every run by nsteps steps in the current mode; the persistent modes
 * synchronise the stream and return HIP if a device-wide barrier timed out in
 * any of the nsteps steps (the states are then undefined).  Every barrier wait
 * is bounded: after a timeout the remaining steps of the call return at once. */
pst_status pst_ensemble_step(pst_ensemble *ens, int nsteps);
/* Test only: polls of a device-wide barrier before it gives up and flags a
 * timeout (default 4194304; 0 makes every barrier that is not already complete
 * time out, so the error path can be exercised with every kernel exiting
 * normally).  INVALID_ARG if polls < 0. */
pst_status pst_ensemble_set_spin_limit(pst_ensemble *ens, long long polls);
pst_status pst_ensemble_set_mode(pst_ensemble *ens, int mode);
/* Current mode (PST_ENS_*), e.g. the one pst_ensemble_autotune picked. */
pst_status pst_ensemble_get_mode(const pst_ensemble *ens, int *mode);

/* Energy of every run (double[nruns]).  Synchronous. */
pst_status pst_ensemble_energy(pst_ensemble *ens, double *per_run);

/* Project every run's state onto divergence-free fields (k = 0 kept). */
pst_status pst_ensemble_project(pst_ensemble *ens);

/* Energy E = 1/2 sum w |uhat|^2 and enstrophy Z = 1/2 sum w |k|^2 |uhat|^2 of
 * every run (double[nruns] each; dE/dt = -2 nu Z without forcing).  Synchronous. */
pst_status pst_ensemble_diagnostics(pst_ensemble *ens, double *energy, double *enstrophy);

/* Relative L2 distance ||a_r - b_r|| / ||b_r|| of every run between two
 * ensembles with the same runs (double[nruns]).  Synchronous on a's stream
 * (b's pending work must be complete). */
pst_status pst_ensemble_rel_l2(pst_ensemble *a, const pst_ensemble *b, double *per_run);

/* Pick the schedule variants (radix order x tile lines) by timing: the
 * persistent kernel's one variant on persistent steps, then, size class by
 * size class, the variant of that class's batched / sequential launches on
 * batched steps (the state is saved and restored around the timing); then, if
 * the ensemble is in one of the two graph modes, switch it to whichever of
 * PERSISTENT_GRAPH and BATCHED_GRAPH steps faster (with one schedule, every
 * mode gives bitwise the same states).  cache_path (may be NULL) is a JSON
 * object keyed by device architecture, precision, RK order and the run sizes
 * (the class variants under the key with "/class<c>" appended, the mode with
 * "/mode"); cached choices are reused unless force != 0.  *chosen (may be
 * NULL) receives the persistent kernel's variant. */
pst_status pst_ensemble_autotune(pst_ensemble *ens, const char *cache_path, int force, int *chosen);
/* One variant (0..3) for the persistent kernel and every class. */
pst_status pst_ensemble_set_schedule(pst_ensemble *ens, int variant);
/* The variant of one size class's batched and sequential launches (class
 * index as in pst_ensemble_query; the persistent modes keep one variant). */
pst_status pst_ensemble_set_class_schedule(pst_ensemble *ens, int cls, int variant);
/* Per class (int[nclasses]): the variants of the batched launches. */
pst_status pst_ensemble_class_schedules(const pst_ensemble *ens, int *variants);

/* Distinct sizes (descending), runs per size, the persistent kernel's variant
 * and grid size.  Arrays need room for 4 entries; any pointer may be NULL. */
pst_status pst_ensemble_query(const pst_ensemble *ens, int *nclasses, int *class_n, int *class_runs,
                              int *variant, int *grid);

/* ------------------------------------------------------------------------
 * Fourier-neural-operator surrogate that advances a velocity field by a
 * fixed number of solver steps (not part of the paper's method; trained on
 * the solver's own trajectories and judged by the solver):
 *   v0 = Wl u + bl;  s_l = Wc_l v_l + bc_l + K_l(v_l);  v_{l+1} = gelu(s_l)
 *   (identity after the last layer);  out = u + Wq2 gelu(Wq1 v_L + bq1) + bq2,
 *   K_l(v) = c2r(R_l . r2c(v) on kx in [0, m), ky, kz in [0, m) U [n-m, n)).
 * Dense channel mixing runs on the matrix cores (BF16 operands, FP32
 * accumulation) unless mfma = 0 (FP32, for gradient checks); the spectral
 * layers run this library's 3D transform kernels.
 * Parameters are one float vector: Wl [w][3], bl [w], per layer Wc [w][w],
 * bc [w], R [(2m)^2 m][w][w][re,im] (modes with kx fastest, then ky, kz each
 * ordered [0, m) then [n-m, n)), then Wq1 [h][w], bq1 [h], Wq2 [3][h], bq2 [3].
 * Fields are float, device, [batch][3][n][n][n] (z, y, x; x fastest).
 * ---------------------------------------------------------------------- */
typedef struct pst_fno pst_fno;

typedef struct {
    int n;       /* grid size (a supported n; n^3 a multiple of 32) */
    int width;   /* channels w of the spectral layers (1..64) */
    int modes;   /* m: retained modes per direction (2 m <= n) */
    int layers;  /* spectral layers (1..8) */
    int hidden;  /* h: projection hidden width (1..256) */
    int batch;   /* maximum batch (1..64, and 2 batch width + width^2 <= 8192 so a
                    mode's spectral mixing fits in 64 KB of LDS); buffers are sized for it */
    int mfma;    /* 1: BF16 matrix-core channel mixing; 0: FP32 */
} pst_fno_params;

pst_status pst_fno_create(const pst_fno_params *p, void *hip_stream, pst_fno **out);
void pst_fno_destroy(pst_fno *fno);
const char *pst_fno_last_error(const pst_fno *fno);
pst_status pst_fno_param_count(const pst_fno *fno, long long *count);

/* Parameters / last gradient as float[count]; set_params also resets Adam. */
pst_status pst_fno_set_params(pst_fno *fno, const float *theta, int mem);
pst_status pst_fno_get_params(pst_fno *fno, float *theta, int mem);
pst_status pst_fno_get_grad(pst_fno *fno, float *grad, int mem);

/* out = surrogate(u) for batch <= p.batch samples (device buffers).  Stream-ordered. */
pst_status pst_fno_forward(pst_fno *fno, const float *u, float *out, int batch);

/* Forward, loss = mean_b ||out_b - tgt_b|| / ||tgt_b|| (written to *loss,
 * double), and the gradient of the loss with respect to every parameter
 * (kept in the object).  Synchronises the stream. */
pst_status pst_fno_loss_grad(pst_fno *fno, const float *u, const float *tgt, int batch, double *loss);

/* One Adam step from the stored gradient (FP32 master weights; the BF16
 * copies used by the matrix cores are refreshed). */
pst_status pst_fno_adam(pst_fno *fno, float lr, float beta1, float beta2, float eps);

/* loss_grad followed by adam(lr, 0.9, 0.999, 1e-8). */
pst_status pst_fno_train_step(pst_fno *fno, const float *u, const float *tgt, int batch, float lr, double *loss);

#ifdef __cplusplus
}
#endif

#endif /* PST_H */
