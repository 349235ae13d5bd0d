/*
 * casclb: cascaded (central-moment) lattice Boltzmann with symmetrized
 * (Strang) operator-split force and source steps, for AMD Instinct MI355X
 * (gfx950).  C ABI.
 *
 * Method (Hajabdollahi & Premnath, arXiv:1806.10247):
 *   per node and time step, fused into one kernel:
 *     pull-stream (eq. 22b / 40b, halfway bounce-back at walls, Sec. 6)
 *     -> output moments rho, j (eq. 24), phi (eq. 42)
 *     -> pre-collision half force step u = (j + F dt/2)/rho (eq. 25, 8A),
 *        half source step phi = phi^o + S dt/2 (eq. 43)
 *     -> cascaded central-moment relaxation (eq. 23 for D2Q9, eq. 41 for the
 *        D2Q5 scalar; the D3Q27 operator is the same central-moment
 *        relaxation extended to the 27-velocity lattice, cf. Appendix A)
 *     -> post-collision half force step as a first-order moment change
 *        (eq. 31: F/6 on D2Q9; F/18 on D3Q27) and half source step as a
 *        zeroth-moment change (eq. 47: S/5)
 *     -> store the post-collision populations (eq. 32, 48).
 *   Solves the Navier-Stokes equations with impressed force F(x,t)
 *   (eq. 11, 13) and the convection-diffusion equation with source S(x,t)
 *   (eq. 33), in lattice units dx = dt = 1 (Sec. 6).
 *
 * Conventions shared by every call:
 *   - Node index n = x + nx*(y + ny*z), x fastest; N = nx*ny*nz.
 *   - Host population arrays are [Q][N] float64, Q = 9 (D2Q9, paper order
 *     of eq. 15), 27 (D3Q27: alpha = d(ex) + 3 d(ey) + 9 d(ez) with
 *     d(0)=0, d(+1)=1, d(-1)=2), and [5][N] for the D2Q5 scalar (paper
 *     order of eq. 34).
 *   - The stored state is the post-collision population f^p after the last
 *     step (the initial state is the equilibrium written by
 *     lb_init_equilibrium).  Step n covers times [n, n+1].
 *   - All calls return LB_OK (0) or a negative LB_E* code; the message of
 *     the last failure is available from lb_last_error.  No call aborts or
 *     throws.  A context is not thread-safe: serialise calls on one context.
 *   - Calls that read results back to the host synchronise the context's
 *     stream; lb_step is asynchronous.
 */
#ifndef CASCLB_H
#define CASCLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_ABI_VERSION 1

/* return codes */
#define LB_OK 0
#define LB_EINVAL (-1)     /* invalid argument or configuration            */
#define LB_ENOMEM (-2)     /* device or host allocation failed             */
#define LB_EHIP (-3)       /* a HIP runtime call failed (no GPU, fault...) */
#define LB_ENONFINITE (-4) /* a residual check found a non-finite value    */
#define LB_ESTATE (-5)     /* call not valid in the context's state        */

/* lattices */
#define LB_D2Q9 0       /* D2Q9 flow (Sec. 4)                             */
#define LB_D2Q9_D2Q5 1  /* D2Q9 flow + D2Q5 passive scalar (Sec. 4, 5)    */
#define LB_D3Q27 2      /* D3Q27 flow                                     */
#define LB_D3Q15 3      /* D3Q15 flow (Appendix A), populations in the
                           order of eq. (A1)                              */

/* per-axis boundary */
#define LB_PERIODIC 0
#define LB_HALFWAY_BB 1 /* no-slip walls half a spacing outside both ends */

/* population storage in device memory */
#define LB_STORE_F64 0      /* float64 deviations, float64 arithmetic          */
#define LB_STORE_F32_DEV 1  /* float32 deviations f - w*rho0, float32 arithmetic */
#define LB_STORE_F16_DEV 2  /* float16 deviations f - w*rho0, float32 arithmetic;
                               stores rounded stochastically (the float16 value
                               above or below, with probabilities in proportion
                               to the distances, so the expected stored value is
                               the float32 one; random bits from a hash of node,
                               population and step, the same for every launch
                               shape) unless LB_FLAG_F16_NEAREST is set          */

/* field element type and location */
#define LB_DTYPE_F64 0
#define LB_DTYPE_F32 1
#define LB_MEM_HOST 0
#define LB_MEM_DEVICE 1

/* time dependence of the force or source: F(x, t) = F(x) * tau(t) */
#define LB_TIME_CONSTANT 0 /* tau = 1                                          */
#define LB_TIME_COS 1      /* tau = cos(omega t); each half step uses the
                              trapezoidal average of tau over that half step
                              (Sec. 6, Womersley flow)                          */

/* which velocity / scalar lb_read_moments returns */
#define LB_MOMENTS_OUTPUT 0      /* u^o = j/rho (eq. 24), phi^o (eq. 42)           */
#define LB_MOMENTS_HALF_FORCED 1 /* u = (j + F/2)/rho (eq. 25), phi^o + S/2 (eq. 43) */

typedef struct lb_ctx lb_ctx;

typedef struct lb_config {
    int32_t abi_version;       /* must be LB_ABI_VERSION                         */
    int32_t lattice;           /* LB_D2Q9, LB_D2Q9_D2Q5, LB_D3Q27, LB_D3Q15      */
    int32_t storage;           /* LB_STORE_*                                     */
    int32_t device;            /* HIP device ordinal                             */
    int64_t nx, ny, nz;        /* lattice size.  2D lattices (no velocity has a z
                                  component): nz > 1 stacks nz independent 2D
                                  lattices (slices z = const), each streamed
                                  and collided on its own; bc[2] is ignored.
                                  Force/source fields, moments and populations
                                  cover all slices; the residual and totals are
                                  sums over all of them                          */
    int32_t bc[3];             /* per axis: LB_PERIODIC or LB_HALFWAY_BB         */
    int32_t residual_interval; /* K: steps between residual checks (0 = none)    */
    double nu;                 /* kinematic viscosity: omega_shear = 1/(3 nu + 1/2)
                                  (omega_4 = omega_5 of eq. 23, Sec. 6); > 0    */
    double omega_bulk;         /* omega_3 (trace of the 2nd-order moments)       */
    double omega_third;        /* 3rd-order moments (omega_6 = omega_7 on D2Q9)  */
    double omega_fourth;       /* 4th and higher order (omega_8 on D2Q9)         */
    double D_phi;              /* scalar diffusivity: omega^phi_1 = omega^phi_2
                                  = 1/(3 D + 1/2) (Sec. 5, 6); > 0 for D2Q9_D2Q5 */
    double omega_phi_high;     /* omega^phi_3 = omega^phi_4                      */
    double rho0;               /* reference density (rest state), > 0            */
    void* stream;              /* hipStream_t the context runs on (NULL: null stream) */
    int64_t plane_pad;         /* elements added between population planes; -1 = auto */
    int32_t block_x;           /* threads per block along x; 0 = auto (64..256, multiple of 64) */
    int32_t flags;             /* LB_FLAG_* bits, 0 by default                   */
    int32_t rows_per_thread;   /* lattice rows each step-kernel thread updates: 1 or 2;
                                  0 = auto.  Only the launch shape changes, results are
                                  bit-identical                                  */
    int32_t x_pairs;           /* x-adjacent nodes each step-kernel thread updates:
                                  1, or 2 (16-bit storage with an even nx, a periodic
                                  x axis and an even plane stride; populations read
                                  and written as 32-bit words; one row per thread);
                                  0 = auto (2 where allowed unless rows_per_thread
                                  is 2 or the lattice is D3Q15, where one node per
                                  thread measured faster).  Only the launch shape
                                  changes, results are bit-identical             */
} lb_config;

/* lb_config.flags */
#define LB_FLAG_EXTERNAL_BUFFERS 1 /* lb_create allocates no population buffers; the
                                      caller must lb_bind_buffers before use      */
#define LB_FLAG_XCD_REMAP 2        /* launch order that hands each of the 8 XCDs a
                                      contiguous range of rows (used when the block
                                      count is a multiple of 8)                   */
#define LB_FLAG_DEBUG_POISON 4     /* debugging aid: before every step lb_step fills
                                      the whole buffer the step writes with NaN bit
                                      patterns (all bytes 0xFF), so a node the step
                                      kernel leaves unwritten shows up as NaN in the
                                      stored state and in the next residual check
                                      (LB_ENONFINITE).  Results are otherwise
                                      unchanged; steps are launched one by one
                                      (no captured step graphs) and cost one more
                                      full-buffer write each                      */
#define LB_FLAG_F16_NEAREST 8      /* float16 storage: round stores to nearest instead
                                      of stochastically.  A per-step change smaller
                                      than half a float16 unit of the stored value is
                                      then lost; lb_set_force_* / lb_set_source_*
                                      refuse (LB_EINVAL) a uniform force or source, or
                                      a field given in host memory, whose largest
                                      per-population change (F / <e_x|e_x> summed
                                      over the axes, S/5) is below half the smallest
                                      float16 subnormal (2^-25), since a lattice
                                      started from rest could not move at all       */

/* Fills *cfg with defaults: D3Q27, F32 deviations, device 0, 64^3 periodic,
 * nu = 1/6, all other rates 1, D_phi = 1/6, rho0 = 1, residual_interval 100,
 * automatic padding and block shape.  Host only, never fails. */
void lb_config_default(lb_config* cfg);

/* Checks a configuration without touching the GPU.  Returns LB_OK or
 * LB_EINVAL and writes a message into msg (msg_len bytes, may be NULL). */
int lb_validate_config(const lb_config* cfg, char* msg, size_t msg_len);

/* Device bytes of one population buffer for cfg (flow planes plus the
 * scalar planes, padded); the context holds two.  0 if cfg is invalid. */
size_t lb_required_bytes(const lb_config* cfg);

/* Creates a context: validates cfg (LB_EINVAL), selects the device and
 * allocates the two population buffers with hipMalloc (LB_ENOMEM / LB_EHIP)
 * unless LB_FLAG_EXTERNAL_BUFFERS is set.
 * The state is undefined until lb_init_equilibrium or lb_write_populations.
 * On failure *out is NULL and lb_last_error(NULL) holds the message. */
int lb_create(lb_ctx** out, const lb_config* cfg);

/* Frees everything the context owns (not bound buffers).  NULL is a no-op. */
void lb_destroy(lb_ctx* ctx);

/* Message of the last failed call on ctx (or of the last failed lb_create
 * when ctx is NULL).  Valid until the next call on the same context. */
const char* lb_last_error(const lb_ctx* ctx);

/* Replaces the population buffers by caller-owned device memory (e.g. from a
 * PyTorch tensor): two distinct buffers of at least lb_required_bytes each,
 * 256-byte aligned.  The caller keeps them alive until lb_destroy; the state
 * must be initialised again afterwards. */
int lb_bind_buffers(lb_ctx* ctx, void* buf_a, void* buf_b, size_t bytes_each);

/* Writes the equilibrium populations of (rho, u, phi) into the stored state
 * and resets the step counter to 0.  Host arrays rho [N], u [dims][N],
 * phi [N]; any may be NULL (rho0, 0, 0).  The flow equilibrium is the
 * product form whose central moments are those of eq. (20) (and its 3D
 * analogue); the scalar equilibrium has the central moments of eq. (39). */
int lb_init_equilibrium(lb_ctx* ctx, const double* rho, const double* u, const double* phi);

/* lb_init_equilibrium from device arrays (same shapes, float64), enqueued on
 * the context's stream without synchronising: the arrays must stay valid
 * until that work has run. */
int lb_init_equilibrium_device(lb_ctx* ctx, const double* rho, const double* u, const double* phi);

/* Moment reset of the stored (post-collision) state, for building the
 * non-equilibrium part that belongs to given moments (a start from estimated
 * fields: alternate single steps with resets to the estimate, then iterate).
 * Every node's populations f (and g) are shifted by f_eq(rho, u) - f_eq(rho_s,
 * u_s) (and g_eq(phi, u) - g_eq(phi_s, u_s)), where rho_s = sum f, u_s =
 * (sum f e) / rho_s and phi_s = sum g are their own moments and f_eq, g_eq the
 * equilibria of lb_init_equilibrium: afterwards the stored state has density
 * rho, momentum rho u and scalar phi, and f - f_eq is unchanged.  Device
 * arrays rho [N], u [dims][N] and, on the scalar lattice, phi [N] (float64,
 * none NULL); enqueued on the context's stream without synchronising.  The
 * step counter is kept; the next residual has no previous velocity.  The
 * paper has no such operation; it prepares the scheme's own iteration.
 * LB_EINVAL for NULL arrays, LB_ESTATE before the state is initialised. */
int lb_reset_moments_device(lb_ctx* ctx, const double* rho, const double* u, const double* phi);

/* Uniform body force (clears any force field).  fz is ignored on 2D lattices. */
int lb_set_force_uniform(lb_ctx* ctx, double fx, double fy, double fz);

/* Spatially varying force: F is [dims][N] of dtype.  mem = LB_MEM_HOST: copied
 * (converted to the arithmetic precision).  mem = LB_MEM_DEVICE: contiguous
 * [dims][N], float64 for LB_STORE_F64; for the float32-arithmetic storages
 * float32 is copied and float64 converted; either way once, into the
 * context's padded layout.  F = NULL removes the field (uniform force applies). */
int lb_set_force_field(lb_ctx* ctx, const void* F, int32_t dtype, int32_t mem);

/* Time dependence of the force: LB_TIME_CONSTANT or LB_TIME_COS with omega. */
int lb_set_force_time(lb_ctx* ctx, int32_t mode, double omega);

/* Uniform source (D2Q9_D2Q5 only, LB_EINVAL otherwise; clears any field). */
int lb_set_source_uniform(lb_ctx* ctx, double s);

/* Source field S [N], same rules as lb_set_force_field (D2Q9_D2Q5 only). */
int lb_set_source_field(lb_ctx* ctx, const void* S, int32_t dtype, int32_t mem);

/* Time dependence of the source (D2Q9_D2Q5 only). */
int lb_set_source_time(lb_ctx* ctx, int32_t mode, double omega);

/* Enqueues nsteps >= 0 time steps on the context's stream (one fused kernel
 * launch per step, plus a reduction every residual_interval steps).  Returns
 * LB_ENONFINITE if a residual check that has already completed found a NaN or
 * infinity (the steps are then not enqueued). */
int lb_step(lb_ctx* ctx, int64_t nsteps);

/* Waits for all work enqueued on the context's stream. */
int lb_synchronize(lb_ctx* ctx);

/* Step counter n (number of steps since the last initialisation). */
int64_t lb_get_step(const lb_ctx* ctx);

/* Sets the step counter (time origin of the force/source factors), e.g. when
 * resuming from populations saved with lb_read_populations. */
int lb_set_step(lb_ctx* ctx, int64_t n);

/* Macroscopic fields of the stored state at the current step: pull, then
 * rho = sum f, u per `kind`, phi per `kind`.  Host outputs rho [N],
 * u [dims][N], phi [N] (phi only for D2Q9_D2Q5); any may be NULL. */
int lb_read_moments(lb_ctx* ctx, int32_t kind, double* rho, double* u, double* phi);

/* lb_read_moments into device arrays (rho [N], u [dims][N], phi [N], any may
 * be NULL), enqueued on the context's stream without synchronising. */
int lb_read_moments_device(lb_ctx* ctx, int32_t kind, double* rho, double* u, double* phi);

/* Stored post-collision populations as full float64 values, f [Q][N],
 * g [5][N] (g may be NULL; ignored unless D2Q9_D2Q5). */
int lb_read_populations(lb_ctx* ctx, double* f, double* g);

/* Overwrites the stored populations (full float64 values, same layout);
 * converted to the storage type.  g may be NULL for flow-only lattices. */
int lb_write_populations(lb_ctx* ctx, const double* f, const double* g);

/* Populations of the box lo[i] <= c_i < lo[i] + ext[i] (coordinates taken
 * modulo the lattice size), f [Q][bn], g [5][bn] with bn = ext0*ext1*ext2,
 * box-local index x + ext0*(y + ext1*z). */
int lb_read_populations_box(lb_ctx* ctx, const int64_t lo[3], const int64_t ext[3], double* f, double* g);

/* Totals of the stored state, accumulated in float64 on the GPU:
 * out[0] = mass sum f, out[1..3] = momentum sum f e, out[4] = scalar sum g. */
int lb_totals(lb_ctx* ctx, double out[5]);

/* lb_totals for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same five totals of the stored state (mass, momentum x/y/z, scalar; float64
 * accumulation) written to out_device, a device pointer to 5 doubles that the
 * caller owns.  Enqueued on the context's stream; does not synchronise and
 * calls no allocating routine.  The partial sums live in a fixed scratch
 * array of the library (1025 records of 10 doubles, about 80 KB per GPU,
 * held until the process ends); every lattice size fits, since at most 1024
 * partial records are formed (grid-stride).  All contexts on one GPU share
 * that array: calls that may overlap in time on one GPU (different streams
 * without ordering between them) race and must not be issued.  The order of
 * the float64 sums differs from lb_totals, so results agree to rounding.
 * LB_EINVAL for a NULL pointer, LB_ESTATE before the state is initialised. */
int lb_totals_noalloc(lb_ctx* ctx, double* out_device);

/* Result of the latest residual check (run by lb_step every
 * residual_interval steps on the step's half-forced velocity u):
 * r = ||u^n - u^{n-K}||_2 / (K ||u^n||_2) (float64 accumulation), +inf for
 * the first check after initialisation; *at_step = step count after the
 * checked step (-1 if none yet); totals (may be NULL) = mass, momentum,
 * scalar of the state that step wrote.  Synchronises. */
int lb_residual(lb_ctx* ctx, double* r, int64_t* at_step, double totals[5]);

/* Walls of 2D lattices (sides of an axis with LB_HALFWAY_BB; axis 0 = x,
 * 1 = y; side 0 = low, 1 = high).  None of them is described in the paper
 * beyond the thermal Couette problem of Sec. 6, which needs all three:
 *
 * lb_set_wall_velocity: the wall moves with (ux, uy) (uz must be 0): a link
 *   pulled from it brings the opposite population plus 6 w_a rho0 (e_a . u_w)
 *   (moving-wall bounce-back, w_a the rest weights).  (0, 0) restores a
 *   resting wall.
 * lb_set_scalar_wall (coupled lattice): fixed != 0 holds the scalar at
 *   `value` on that wall by anti-bounce-back,
 *   g_a = -g^p_opp(a) + value (1/3 + u_w,k^2) + 2 S_tot/5 (k the axis of a;
 *   the last term restores the source share the collision gave the
 *   reflected population); fixed = 0 restores the no-flux (bounce-back) wall.
 * lb_set_viscous_heating (coupled lattice): adds c_h (S:S) to the scalar
 *   source of every node and step, S the flow's strain-rate tensor from the
 *   non-equilibrium second moments of the streamed populations:
 *   S_xy = -3 w_shear/(2 rho0) Pi_xy (as printed),
 *   S_xx -+ S_yy from Pi_xx -+ Pi_yy with w_shear (difference) and w_bulk
 *   (sum), Pi_ab = sum f e_a e_b - rho u_a u_b - rho/3 delta_ab.  For a
 *   specific heat C_v, c_h = 2 nu / C_v.  0 turns it off.
 * All take effect from the next lb_step; LB_EINVAL for a periodic axis, a 3D
 * lattice or (scalar settings) a lattice without a scalar. */
int lb_set_wall_velocity(lb_ctx* ctx, int32_t axis, int32_t side, double ux, double uy, double uz);
int lb_set_scalar_wall(lb_ctx* ctx, int32_t axis, int32_t side, int32_t fixed, double value);
int lb_set_viscous_heating(lb_ctx* ctx, double coefficient);

/* Velocity-dependent x-force of 2D lattices: the force on every node becomes
 * F_x - s u_x, F the uniform force or field, as the Lorentz force -sigma B0^2
 * u_x of a transverse magnetic field (Hartmann flow, Sec. 6; s = sigma B0^2).
 * Sec. 6 notes that such a force makes the force step an implicit equation for
 * u; it is taken as the implicit midpoint rule, as in the batched solver below:
 * rho u_x = j_x + (F_pre,x - s u_x)/2 before the collision (LB_MOMENTS_HALF_FORCED
 * reads this u_x), momentum change F_tot,x - s u_x over the step.  s >= 0; 0
 * (the default) turns it off.  LB_EINVAL on a 3D lattice or a bad s. */
int lb_set_lorentz(lb_ctx* ctx, double s);

/* Scalar residual of the same check on the coupled lattice (LB_D2Q9_D2Q5):
 * r_phi = ||phi^n - phi^{n-K}||_2 / (K ||phi^n||_2) of the half-sourced
 * scalar phi* = phi^o + S_pre/2 (eq. 43), float64 accumulation; +inf until
 * two checks have run.  LB_EINVAL on a lattice without a scalar.
 * Synchronises. */
int lb_residual_scalar(lb_ctx* ctx, double* r_phi);

typedef struct lb_info {
    int64_t nodes;           /* N                                            */
    int32_t q;               /* flow populations per node                    */
    int32_t q_scalar;        /* scalar populations per node (0 or 5)         */
    int64_t plane_stride;    /* elements between population planes           */
    int32_t elem_bytes;      /* bytes per stored population                  */
    int32_t block_x;         /* threads per block of the step kernel         */
    double bytes_per_update; /* algorithmic HBM bytes per lattice update      */
    void* buf_current;       /* device buffer holding the stored state        */
    void* buf_other;         /* the second buffer                             */
    const char* step_kernel; /* name of the step kernel                       */
} lb_info;

/* Layout and cost figures of a context (host only). */
int lb_get_info(const lb_ctx* ctx, lb_info* info);

/* Streaming copy kernel (measurement aid for the HBM roofline): copies
 * `bytes` (multiple of 16) from src to dst, both device pointers, on stream. */
int lb_stream_copy(void* dst, const void* src, size_t bytes, void* stream);

/* Streaming kernels for the HBM ceiling (measurement aid): mode 0 copies
 * `bytes` from src to dst, mode 1 reads src (folding what it loads into one
 * `width`-byte vector per block, written to dst, which must hold that many),
 * mode 2 writes zeros to dst; non-temporal `width`-byte (8 or 16) vectors,
 * 4 per thread per pass; blocks = 0: one pass of 1024-vector blocks, > 0: a
 * grid-stride loop over that many 256-thread blocks.  bytes a multiple of 16,
 * device pointers, on `stream`.  LB_EINVAL for bad arguments. */
int lb_stream_bench(void* dst, const void* src, size_t bytes, int32_t mode, int32_t width, int64_t blocks,
                    void* stream);

/* ------------------------------------------------------------------------ */
/* Batched independent channels (parameter sweeps)                            */
/* ------------------------------------------------------------------------ */
/*
 * Many independent D2Q9 channels, each periodic in x with halfway
 * bounce-back walls at both ends of y, driven by a uniform force F_b along x
 * and retarded by the velocity-dependent Lorentz force -s u_x of a transverse
 * magnetic field (Hartmann flow, Sec. 6; s = sigma B0^2 = Ha^2 rho nu / L^2).
 * The paper notes that a velocity-dependent force makes the force step
 * (eq. 13) an implicit equation for u; both half steps are taken as the
 * implicit midpoint rule: rho u_x = j_x + (F_b - s u_x)/2 before collision,
 * momentum change F_b - s u_x over the step.  The cascaded collision and the
 * half steps are those of the single-lattice D2Q9 update.
 *
 * One call of lb_batch_run is one persistent kernel launch (replayed from a
 * captured HIP graph): workgroups take domains from a work queue and step
 * each to its steady residual r = ||u^n - u^{n-K}|| / (K ||u^n||) < tol
 * (half-forced velocity, float64 reduction), keeping a domain in LDS when its
 * two population buffers fit; finished domains retire.
 */
typedef struct lb_batch lb_batch;

typedef struct lb_batch_domain {
    int32_t nx, ny;  /* nodes; nx >= 1, ny >= 1, nx * ny <= 2^20        */
    double nu;       /* kinematic viscosity > 0                          */
    double force_x;  /* F_b                                              */
    double lorentz;  /* s >= 0                                           */
} lb_batch_domain;

typedef struct lb_batch_config {
    int32_t abi_version;     /* LB_ABI_VERSION                                  */
    int32_t storage;         /* LB_STORE_F64 or LB_STORE_F32_DEV               */
    int32_t device;          /* HIP device ordinal                              */
    int32_t check_interval;  /* K >= 1: steps between residual checks           */
    double rho0;             /* rest density > 0                                */
    double omega_bulk, omega_third, omega_fourth;  /* in (0, 2), as lb_config */
    void* stream;            /* hipStream_t; NULL: the batch creates its own    */
    int32_t block;           /* threads per workgroup (64..1024, multiple of 64); 0 = 512 */
    int32_t lds_policy;      /* 0: LDS-resident domains where they fit; 1: never */
    int32_t lds_bytes;       /* LDS per workgroup for resident domains; 0 = auto */
    int32_t routed;          /* 0..ndomains: the domains of longest expected
                                time in the persistent launch (the steps their
                                slowest mode needs times a step's time on one
                                workgroup) are stepped instead by ordinary
                                launches, one per step over all of them, each
                                domain tiled over 256-node workgroups, on a
                                stream of the batch's own driven by a host
                                thread, with the same stopping rule, while the
                                persistent launch runs the rest; 0 = none       */
    int32_t routed_cus;      /* with routed > 0: compute units the persistent
                                launch leaves to the routed launches (its grid
                                covers the others); 0 = none.  Must be >= 0 and,
                                with routed > 0, below the device's count
                                (LB_EINVAL otherwise); unused when routed = 0   */
} lb_batch_config;

/* lb_batch_domain status values */
#define LB_BATCH_NOT_RUN 0
#define LB_BATCH_CONVERGED 1   /* r < tol                                       */
#define LB_BATCH_STATIONARY 2  /* u did not change at all in K steps (storage precision) */
#define LB_BATCH_MAX_STEPS 3   /* step limit reached                            */
#define LB_BATCH_NONFINITE 4   /* NaN or infinity                               */

void lb_batch_config_default(lb_batch_config* cfg);

/* Validates, allocates the population pools (two buffers per domain) and
 * copies the domain table (ndomains >= 1).  State undefined until
 * lb_batch_init.  On failure *out is NULL, lb_batch_last_error(NULL) says why. */
int lb_batch_create(lb_batch** out, const lb_batch_config* cfg, const lb_batch_domain* domains, int32_t ndomains);
void lb_batch_destroy(lb_batch* b);
const char* lb_batch_last_error(const lb_batch* b);

/* Every domain to the rest state (rho0, u = 0); clears the results. */
int lb_batch_init(lb_batch* b);

/* Continues every domain from its stored state for at most max_steps steps
 * (>= 1) or until r < tol, in one persistent launch; asynchronous (routed
 * domains are stepped by a host thread that the next call on the batch
 * joins). */
int lb_batch_run(lb_batch* b, int64_t max_steps, double tol);

/* Per-domain results of the last run (arrays of ndomains; any may be NULL):
 * steps taken, last residual (+inf if fewer than two checks), status.
 * Synchronises. */
int lb_batch_results(lb_batch* b, int64_t* steps, double* residual, int32_t* status);

/* Density [ny][nx] and half-forced velocity [2][ny][nx] of one domain. */
int lb_batch_read_moments(lb_batch* b, int32_t domain, double* rho, double* u);

/* Stored post-collision populations of one domain, full float64 values,
 * [9][ny][nx] in the order of eq. (15). */
int lb_batch_read_populations(lb_batch* b, int32_t domain, double* f);
int lb_batch_write_populations(lb_batch* b, int32_t domain, const double* f);

/* Autotuner: times `sample_steps` steps of every domain for each workgroup
 * size in {256, 512, 1024} with and without LDS residency (the state is
 * saved and restored), keeps the fastest and reports it. */
int lb_batch_autotune(lb_batch* b, int64_t sample_steps, int32_t* block, int32_t* lds_policy, double* best_ms);

#ifdef __cplusplus
}
#endif

#endif /* CASCLB_H */
