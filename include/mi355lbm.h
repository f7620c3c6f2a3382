/*
 * mi355lbm.h -- C ABI of the MI355X (gfx950) cumulant lattice Boltzmann
 * solver and Fourier neural operator surrogate.
 *
 * The solver advances the D3Q27 cumulant lattice Boltzmann method on a 3D
 * obstructed channel (paper Sec. 3.1-3.2): velocity inlet at x = -1/2,
 * zero-gradient (extrapolation) outlet, no-slip lateral walls, halfway or
 * linearly interpolated bounce-back at the obstacle, cumulant collision with
 * the optional fourth-order parametrised mode and third-order limiter.  It
 * records running means of u, v, w, p, snapshots and the force on the object
 * (paper Sec. 2, data capture).  The surrogate is the 3D Fourier neural
 * operator of paper Sec. 4 / App. A.2, predicting mean fields from geometry
 * and Reynolds number.
 *
 * Conventions
 *  - Lattice direction i = 9(cz+1) + 3(cy+1) + (cx+1), opposite 26 - i,
 *    weights w = W(cx)W(cy)W(cz) with W(0) = 2/3, W(+-1) = 1/6.
 *  - Fields use the natural layout [k][nz][ny][nx] with x fastest; N =
 *    nx*ny*nz.  Populations are exchanged as shifted values fbar = f - w_i.
 *  - Every call returns 0 (LBM_OK) or a positive error code; no call aborts
 *    or throws.  lbm_last_error() gives the message of the last failure.
 *  - Host pointers and device pointers are told apart by an explicit flag
 *    argument where both are accepted; device pointers must be allocated on
 *    the device the object was created on.
 *  - All device work of an object is enqueued on the HIP stream given at
 *    creation (NULL = the null stream).  Calls that return host data
 *    synchronise that stream; lbm_step and fno_forward do not.
 *  - The caller owns every buffer it passes; the library owns the
 *    populations, accumulators, tables and workspaces it allocates, and
 *    frees them in the destroy call.
 *  - Objects are not thread-safe: one host thread at a time per object.
 */
#ifndef MI355LBM_H
#define MI355LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_OK = 0,
  LBM_EINVAL = 1,    /* bad argument (shape, pointer, parameter range)          */
  LBM_ENOMEM = 2,    /* device or host allocation failed                         */
  LBM_EDEVICE = 3,   /* HIP runtime error; sticky                                */
  LBM_EUNSTABLE = 4, /* run diverged: a check step (lbm_params.check_every) found
                        a cell with non-finite or out-of-range density or speed,
                        or lbm_mass found a non-finite mass; sticky              */
  LBM_ESTATE = 5     /* call not valid in the object's state                     */
};

/* Storage of the shifted populations fbar = f - w_i.  Collision arithmetic is
 * FP64 for LBM_F64 and FP32 otherwise; means and forces are FP64 always.    */
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2, LBM_BF16S = 3 };

/* Collision mode (paper Sec. 3.2): plain cumulant (orders >= 3 relaxed to
 * zero) or the fourth-order parametrised operator with limiter, which the
 * paper switches off below Re_c = 3000.  AUTO picks K17 iff
 * u_in * ny / nu >= 3000 (Reynolds number on the channel height).            */
enum { LBM_MODE_AUTO = -1, LBM_MODE_PLAIN = 0, LBM_MODE_K17 = 1 };

typedef struct lbm_sim lbm_sim;

typedef struct {
  int32_t nx, ny, nz;      /* cells; nx % 64 == 0, ny % 2 == 0, nz >= 1          */
  int32_t storage;         /* LBM_F64 .. LBM_BF16S                                */
  int32_t periodic[3];     /* 1: periodic axis.  0: x has the inlet (x = -1/2)
                              and the outlet (x = nx - 1/2); y, z have no-slip
                              walls at -1/2 and n - 1/2                           */
  double u_in;             /* inlet velocity along +x, lattice units              */
  double nu;               /* lattice viscosity; omega1 = 1/(3 nu + 1/2); ignored
                              when re > 0                                         */
  double omega2;           /* bulk relaxation rate (1.0)                          */
  int32_t mode;            /* LBM_MODE_*                                          */
  int32_t galilean;        /* 1: Galilean correction of the 2nd-order rates       */
  double lambda;           /* third-order limiter of the K17 mode (0.01)          */
  int32_t obstacle_bc;     /* 0 halfway bounce-back, 1 linear interpolated (q)    */
  double body_force[3];    /* uniform body force (0 for the channel)              */
  int64_t avg_start;       /* step index from which the mean is sampled; <0 off   */
  int32_t snap_every;      /* snapshot period in steps (0 = no snapshots)         */
  int32_t snap_count;      /* ring of the last snap_count snapshots               */
  int64_t snap_start;      /* first step index eligible for a snapshot            */
  int32_t force_every;     /* record the obstacle force every k steps (0 = off)   */
  int32_t xcd_remap;       /* 1: map workgroups to XCD-contiguous tiles           */
  uint64_t perturb_seed;   /* when u0 is NULL and perturb_amp != 0, the initial
                              velocity of fluid cell n, component d, is
                              perturb_amp * xi(seed, 3n + d), xi the uniform
                              [-1, 1) variate of counter-based SplitMix64
                              (output k = mix(seed + (k+1) * 0x9E3779B97F4A7C15),
                              top 53 bits), generated on the device            */
  double perturb_amp;
  double re;               /* > 0: Reynolds number on l_ref (paper Sec. 3.1, Re
                              set through the viscosity): nu = u_in l_ref / re;
                              needs u_in > 0.  0: take nu as given               */
  double l_ref;            /* reference length in cells for re; <= 0: ny, the
                              channel height                                      */
  int32_t check_every;     /* > 0: every check_every-th step (steps k, 2k, ...)
                              flags, on the device, any fluid cell whose
                              pre-collision density leaves (0, 2) or whose speed
                              reaches the lattice sound speed 1/sqrt(3), NaN and
                              infinity included; the flag travels to the host
                              asynchronously and the next call on the object
                              returns the sticky LBM_EUNSTABLE.  0: off         */
  int32_t reserved;        /* 0                                                   */
  int64_t force_capacity;  /* > 0: the force series is a ring holding the last
                              force_capacity samples (required with a caller
                              workspace); 0: it grows without bound              */
} lbm_params;

/* Fill *p with defaults (F32, channel, omega2 = 1, Galilean on, lambda 0.01,
 * halfway bounce-back, averaging from step 0, no snapshots, forces every
 * step, XCD remap on, no stability check, growing force series, nu for
 * Re 5000 on the channel height, re = 0) for an nx x ny x nz grid.          */
int lbm_default_params(lbm_params* p, int32_t nx, int32_t ny, int32_t nz);

/* Create a solver (paper Sec. 3.1: obstacle in a channel, inlet velocity u_in,
 * Re set through the lattice viscosity).
 *  solid      host uint8 [N], 1 = obstacle cell (NULL: no obstacle).  The
 *             obstacle must keep 3 cells clear of inlet and outlet.
 *  nlinks, link_cell, link_dir, link_q
 *             host arrays: wall-distance fractions q in (0, 1] for links from
 *             fluid cell link_cell along direction link_dir into the obstacle
 *             (paper Sec. 3.2, interpolated bounce-back); links not listed
 *             take q = 1/2.  Ignored for halfway bounce-back.  May be 0/NULL.
 *  u0         host double [3][N] initial velocity (NULL: rest); the initial
 *             state is the equilibrium at rho = 1 and u0.
 *  hip_stream hipStream_t cast to void* (NULL: null stream).
 * On success *out owns device memory of about 2*27*N*sizeof(storage) bytes
 * (two population lattices) plus 32 B per cell when averaging is on.
 * Errors: LBM_EINVAL for a grid the kernels do not tile, a non-positive
 * viscosity, omega2 outside (0, 2), an obstacle within 3 cells of inlet or
 * outlet, links out of range, and the fourth-order mode where its rates are
 * undefined (|omega1 - omega2| < 1e-3, where A and B have a pole, or
 * omega3..5 outside (0, 2)); LBM_ENOMEM; LBM_EDEVICE.                       */
int lbm_create(const lbm_params* p, const uint8_t* solid, int64_t nlinks, const int64_t* link_cell,
               const uint8_t* link_dir, const double* link_q, const double* u0, void* hip_stream, lbm_sim** out);

/* Device bytes that lbm_create_in needs as a caller workspace for these
 * parameters and this solid mask (host uint8 [N] or NULL): two population
 * lattices in the padded layout, cell flags, boundary tables, force partials, FP64
 * accumulators when averaging, the snapshot ring, the force ring
 * (force_capacity samples) and a stability flag.  Host work only; no device
 * call.  Errors: LBM_EINVAL, as lbm_create would return it.                  */
int lbm_workspace_size(const lbm_params* p, const uint8_t* solid, size_t* bytes);

/* lbm_create with an optional caller workspace: d_workspace NULL behaves as
 * lbm_create; otherwise it is device memory of at least
 * lbm_workspace_size() bytes, 256-byte aligned, on the current device, that
 * the caller owns and keeps alive until lbm_destroy, which does not free it.
 * All state the step touches then lives in it; with forces on, the force
 * series must be a ring (force_capacity > 0).  Creation still allocates and
 * frees small temporaries (link cells, u0) and readouts into host pointers
 * stage through temporaries; lbm_step allocates nothing.
 * Errors: LBM_EINVAL (workspace too small or misaligned, force_capacity 0
 * with forces on, and everything lbm_create rejects), LBM_ENOMEM,
 * LBM_EDEVICE.                                                              */
int lbm_create_in(const lbm_params* p, const uint8_t* solid, int64_t nlinks, const int64_t* link_cell,
                  const uint8_t* link_dir, const double* link_q, const double* u0, void* d_workspace,
                  size_t workspace_bytes, void* hip_stream, lbm_sim** out);

/* Advance nsteps steps (asynchronous on the object's stream).  One step is
 * one time step of the method of paper Sec. 3.1-3.2: streaming of the 27
 * populations with the channel's boundary rules (velocity inlet, zero-
 * gradient outlet, no-slip walls, bounce-back at the obstacle) and the
 * cumulant collision; plus the data capture of Sec. 2 (running means,
 * snapshots, force on the object) when due.  It is one fused
 * stream-and-collide launch (two-lattice pull: the step reads the previous
 * post-collision populations at the upstream cells from one lattice and
 * writes its own to the other), a force reduction when a force sample is due, and a 4-byte
 * copy of the stability flag after a check step.  nsteps = 0 only reports
 * the object's state (LBM_EUNSTABLE once a finished check step has flagged).
 * Errors: LBM_EINVAL (negative count), the sticky LBM_EUNSTABLE and
 * LBM_EDEVICE, LBM_ENOMEM (growing force series).                            */
int lbm_step(lbm_sim* s, int64_t nsteps);

/* Mean fields (paper Sec. 2: mean velocity and pressure).  out is [4][N]
 * double (u, v, w, p = (rho - 1)/3) averaged over the sampled steps, zero in
 * solid cells; out_on_device selects a device or host pointer.  *nsamples
 * receives the number of sampled steps.  Synchronises.                       */
int lbm_mean_fields(lbm_sim* s, double* out, int out_on_device, int64_t* nsamples);

/* Mean fields pooled for the surrogate (paper Sec. 2: fields stored at a
 * reduced resolution; App. A.2: 128x64x64 training fields, augmented by 90
 * degree turns about the x axis).  d_out is device float [4][X][Y][Z]
 * (u, v, w, p; Z fastest) with X = nx/factor, Y = ny/factor, Z = nz/factor:
 * each value is the mean over a factor^3 block of the values lbm_mean_fields
 * returns (solid cells count as 0).  quarter_turns in 0..3 turns the pooled
 * field about +x: the value at (x, y, z) is R^q u(R^-q (x, y, z)) with R
 * taking +y to +z and +z to -y (requires ny == nz).  The caller owns d_out.
 * Errors: LBM_EINVAL (factor does not divide the grid, turns out of range),
 * LBM_ESTATE (averaging off).  Asynchronous on the object's stream.          */
int lbm_mean_fields_pooled(lbm_sim* s, int32_t factor, int32_t quarter_turns, float* d_out);

/* Snapshots (paper Sec. 2: 20 snapshots 25 steps apart).  out is
 * [k][4][N] float (u, v, w, p), oldest first, k = min(taken, snap_count)
 * written to *k; steps[j] (host int64, may be NULL) receives the step index
 * of snapshot j.  Synchronises.                                              */
int lbm_snapshots(lbm_sim* s, float* out, int out_on_device, int32_t* k, int64_t* steps);

/* Force on the obstacle (paper Sec. 2: forces in x and y; all three given).
 * Host double [n][3], the retained samples in step order (all of them, or
 * the last force_capacity of a ring); *n receives their number; the step
 * index of sample j is returned in steps[j] when steps is not NULL.  Force of step n:
 * sum over fluid->obstacle links (x, j) of c_j (f_jbar(x) entering step n
 * + f*_j(x) leaving it).  Synchronises.                                      */
int lbm_forces(lbm_sim* s, double* fxyz, int64_t cap, int64_t* n, int64_t* steps);

/* Instantaneous (u, v, w, p) of the current state, float [4][N].            */
int lbm_moments(lbm_sim* s, float* out, int out_on_device);

/* Current pre-collision populations, natural layout, double fbar [27][N]
 * (solid cells 0): the populations the next step collides, boundary rules
 * applied.  Host pointer.  Synchronises.                                    */
int lbm_get_populations(lbm_sim* s, double* fbar);

/* The same for the cells of one box [x0, x0 + bx) x [y0, y0 + by) x
 * [z0, z0 + bz): host double fbar [27][bz][by][bx].  LBM_EINVAL for a box
 * not inside the grid.  Synchronises.  For checking sampled cells of grids
 * whose full state does not fit the host.                                   */
int lbm_get_populations_box(lbm_sim* s, int32_t x0, int32_t y0, int32_t z0, int32_t bx, int32_t by, int32_t bz,
                            double* fbar);

/* Replace the state with natural-layout fbar [27][N] (host double, rounded
 * to the storage type), read in place by the next step; keeps step count and
 * accumulators.                                                              */
int lbm_set_populations(lbm_sim* s, const double* fbar);

/* Sum of rho - 1 over fluid cells (FP64) of the current state; sets the
 * sticky LBM_EUNSTABLE state if it is not finite.  Synchronises.             */
int lbm_mass(lbm_sim* s, double* mass);

/* Raw checkpoint: populations in storage layout plus step count, state kind,
 * accumulators and snapshot ring.  lbm_export_state with blob == NULL
 * reports the size in *used.  Restoring into an object created with the
 * same parameters and geometry continues bitwise identically.               */
int lbm_export_state(lbm_sim* s, void* blob, size_t cap, size_t* used);
int lbm_import_state(lbm_sim* s, const void* blob, size_t n);

/* Step counter, omega1 and the resolved mode.                                */
int lbm_info(const lbm_sim* s, int64_t* steps, double* omega1, int32_t* mode);

/* Kernel timing with HIP events on the object's stream: while enabled, every
 * stream-and-collide launch is bracketed by events; lbm_profile_read returns
 * the summed elapsed milliseconds and the number of launches (synchronises)
 * and resets the counters.                                                   */
int lbm_profile(lbm_sim* s, int enable);
int lbm_profile_read(lbm_sim* s, double* total_ms, int64_t* launches);

/* Bandwidth probe (measurement support for the roofline of lbm_step, not
 * a step of the method): `passes` launches of a kernel that moves exactly
 * the step's memory traffic, every cell's 27 populations loaded from the
 * upstream cells of the current lattice and stored to the cell in the
 * other lattice, with the step kernel's addressing, tile order and cache
 * hints, with no collision.  2 * 27 * sizeof(storage) bytes per cell per
 * pass.  The current lattice is only read, so the state is unchanged;
 * passes must be even (kept for callers of earlier versions).
 * *ms_per_pass receives the event-timed average.  Synchronises.
 * Errors: LBM_EINVAL (null pointer, odd or non-positive passes),
 * LBM_EDEVICE.                                                             */
int lbm_bandwidth_probe(lbm_sim* s, int32_t passes, double* ms_per_pass);

/* Plain-copy bandwidth (measurement support, not a step of the method): a
 * device-to-device copy of `bytes` (a multiple of 16) between two buffers
 * the call allocates and frees, one 16-byte vector per lane with
 * non-temporal stores, run `passes` times after two warm-up passes on
 * hip_stream; *ms_per_pass receives the event-timed average (read + write =
 * 2 * bytes per pass).  The attainable-bandwidth reference next to the
 * roofline of lbm_step.  Synchronises.  Errors: LBM_EINVAL, LBM_ENOMEM,
 * LBM_EDEVICE.                                                             */
int lbm_copy_bandwidth(int64_t bytes, int32_t passes, void* hip_stream, double* ms_per_pass);

void lbm_destroy(lbm_sim* s);
const char* lbm_last_error(const lbm_sim* s); /* s may be NULL: global error */

/* ------------------------------------------------------------------------ */
/* Fourier neural operator (paper Sec. 4 and App. A.2): lifting 4 -> width,
 * `layers` Fourier layers (truncated 3D real DFT keeping kx, ky in
 * {0..m-1, -m..-1} and kz in {0..m-1}, per-mode complex channel mixing,
 * truncated inverse DFT, plus a pointwise linear map and bias, GELU after
 * all but the last), projection width -> proj_hidden (GELU, or the sine of
 * a SIREN) -> cout.
 * arch = 1 gives the hybrid F/FNO of App. A.2 instead: every layer is the
 * residual block v + W2 GELU(W1 s + b1) + b2 around the same spectral
 * convolution s of v (width -> ff_hidden -> width), with no pointwise map
 * beside it and no activation on the residual stream.
 * arch = 2 gives the factorized FNO of Table 2 (per-axis layers after Tran
 * et al.): the hybrid's residual block with s the sum over the three axes of
 * 1D spectral convolutions, each a real DFT along the axis truncated to
 * modes k = 0..m-1 (m = mx, my or mz), per-mode complex channel mixing and
 * the c2r inverse along the axis (1/n, modes k >= 1 counted twice).
 * Contractions run as BF16 MFMA with FP32 accumulation.                      */
typedef struct fno_net fno_net;

typedef struct {
  int32_t nx, ny, nz;       /* grid; powers of two, nx*ny*nz % 8192 == 0      */
  int32_t cin, cout;        /* input / output channels (4, 4)                 */
  int32_t width;            /* channels of the Fourier layers (32), % 16 == 0,
                               at most 64                                     */
  int32_t layers;           /* Fourier layers (4)                             */
  int32_t mx, my, mz;       /* retained modes (16): powers of two, 2m <= n;
                               2*my*mz >= 32 (>= 16 when width > 32); the
                               factorized FNO's modes per axis, 4 to 16     */
  int32_t proj_hidden;      /* projection hidden width (128), % 16 == 0       */
  int32_t max_batch;        /* largest batch the workspaces are sized for     */
  int32_t proj_act;         /* projection hidden activation: 0 GELU (erf),
                               1 sine (SIREN, App. A.2): sin(proj_w0 (W1 v + b1))
                               with Sitzmann's initialisation; the sine needs
                               proj_hidden <= 128, width <= 64, cout <= 16   */
  float proj_w0;            /* SIREN frequency (30); ignored for GELU         */
  int32_t arch;             /* 0 FNO, 1 hybrid F/FNO, 2 factorized FNO; the
                               hybrid needs width <= 32, nz in [16, 256],
                               2*mz <= 32 and ff_hidden <= 128; the
                               factorized FNO width 16 or 32, nz in
                               [32, 256] and ff_hidden <= 128               */
  int32_t ff_hidden;        /* feed-forward width of the hybrid and the
                               factorized FNO (128), % 16 == 0; ignored for
                               the FNO                                        */
} fno_params;

/* Parameter vector layout (FP32, fno_param_count entries), in this order:
 * lift W [width][cin], lift b [width]; per layer l: spectral weights
 * [2*mx][2*my][mz][width_in][width_out][2] (re, im) (factorized FNO: the
 * axis weights [mx][width_in][width_out][2], then [my][...], then [mz][...]),
 * then for the FNO the pointwise W [width][width] (out, in) and bias
 * [width], for the hybrid and the factorized FNO W1 [ff_hidden][width],
 * b1 [ff_hidden], W2 [width][ff_hidden], b2 [width];
 * proj W1 [proj_hidden][width], b1 [proj_hidden], W2 [cout][proj_hidden],
 * b2 [cout].                                                                 */
int64_t fno_param_count(const fno_params* p);

/* Create with parameters initialised from seed (uniform fan-in scaling);
 * allocates the BF16 working copy, FP32 master copy, Adam moments and the
 * activation workspaces for max_batch.                                       */
int fno_create(const fno_params* p, uint64_t seed, void* hip_stream, fno_net** out);

/* Copy the FP32 parameter vector in or out (host pointers).                  */
int fno_set_params(fno_net* n, const float* host_params, int64_t count);
int fno_get_params(fno_net* n, float* host_params, int64_t count);

/* Forward pass: x device BF16 (uint16 bit patterns) [B][cin][nx][ny][nz]
 * (z fastest), y device FP32 [B][cout][nx][ny][nz].  Asynchronous.           */
int fno_forward(fno_net* n, const uint16_t* x, int32_t B, float* y);

/* Loss and gradients: masked mean squared error over cells where mask != 0
 * (device uint8 [nx][ny][nz], shared by all samples and channels); target
 * device FP32 [B][cout][nx][ny][nz].  Gradients land in the FP32 gradient
 * buffer; host_grads (may be NULL) receives a copy; *loss (host, may be
 * NULL) the loss.  Asynchronous unless a host output is requested, then it
 * synchronises.  An empty mask gives zero gradients, and LBM_EINVAL when the
 * loss is requested.                                                         */
int fno_loss_grad(fno_net* n, const uint16_t* x, const float* target, const uint8_t* mask, int32_t B,
                  float* loss, float* host_grads);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the gradients of the
 * last fno_loss_grad call with learning rate lr.                             */
int fno_adam_step(fno_net* n, float lr);

/* fno_loss_grad followed by fno_adam_step.                                   */
int fno_train_step(fno_net* n, const uint16_t* x, const float* target, const uint8_t* mask, int32_t B, float lr,
                   float* loss);

/* Per-field min-max scaling of the surrogate's data (App. A.2: min-max
 * scaling applied to each field).  x is device float [S][C][P], C <= 16.
 * fno_field_minmax writes the minimum and maximum of each channel over all
 * samples and points to host lo[C], hi[C] and synchronises hip_stream.
 * fno_field_scale maps x in place to (x - lo[c]) / (hi[c] - lo[c]) (a
 * channel with hi == lo maps to 0), or with inverse != 0 back to
 * x (hi[c] - lo[c]) + lo[c]; lo, hi are host arrays; asynchronous.
 * Errors: LBM_EINVAL (null pointer, sizes), LBM_ENOMEM, LBM_EDEVICE.        */
int fno_field_minmax(const float* x, int64_t S, int32_t C, int64_t P, void* hip_stream, float* lo, float* hi);
int fno_field_scale(float* x, int64_t S, int32_t C, int64_t P, const float* lo, const float* hi, int32_t inverse,
                    void* hip_stream);

/* fno_field_minmax for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result, with the per-block partials in a fixed device array of the
 * library (4 MiB per GPU, held until the process ends) instead of a
 * temporary allocation.  It calls no allocating routine.  Limit:
 * S * ceil(P / 4096) * C <= 524288 (e.g. 512 samples of 4 fields of
 * 128x64x64), larger inputs return LBM_EINVAL.  Every call on one GPU
 * shares that GPU's array and overwrites what it reads, so calls that
 * overlap on one GPU (several host threads or streams) race; serialise
 * them.  Synchronises hip_stream.  Errors: LBM_EINVAL, LBM_EDEVICE.        */
int fno_field_minmax_noalloc(const float* x, int64_t S, int32_t C, int64_t P, void* hip_stream, float* lo,
                             float* hi);

void fno_destroy(fno_net* n);
const char* fno_last_error(const fno_net* n);

/* ------------------------------------------------------------------------ */
/* 3D U-Net surrogate (paper Sec. 4, Table 2; architecture of App. A.2): a
 * 3D encoder-decoder with skip connections on the same inputs and outputs
 * as the Fourier operator.  Encoder: four stages of widths widths[0..3],
 * each two blocks of 3x3x3 convolution (one cell of zero padding, no bias),
 * batch normalisation and ReLU, then 2x2x2 max pooling.  Bottleneck: two
 * blocks of `bottleneck` channels.  Decoder: trilinear upsampling by two
 * (half-pixel centres, clamped at the faces), concatenation with the skip
 * connection of the same level (upsampled channels first), two blocks.
 * Head: 1x1x1 convolution with bias to cout channels and a sigmoid.
 * Batch normalisation uses the batch statistics (biased variance,
 * eps 1e-5) in training passes, which also move the running statistics
 * 10% of the way (unbiased variance); evaluation passes use the running
 * statistics.  Convolutions run as BF16 MFMA with FP32 accumulation;
 * batch-norm statistics and reductions in FP64.                            */
typedef struct unet_net unet_net;

typedef struct {
  int32_t nx, ny, nz;       /* grid; positive multiples of 16                  */
  int32_t cin, cout;        /* input / output channels, 1..8 (4, 4)            */
  int32_t widths[4];        /* encoder widths (32, 64, 128, 256); powers of
                               two in [8, 2048]                               */
  int32_t bottleneck;       /* bottleneck width (512); power of two <= 2048    */
  int32_t max_batch;        /* largest batch the workspaces are sized for     */
} unet_params;

/* Parameter vector layout (FP32, unet_param_count entries): per block in
 * forward order (enc0a, enc0b, ..., enc3b, bottleneck a, b, dec3a, dec3b, ...,
 * dec0a, dec0b) the convolution weight [out][in][27] (tap
 * t = 9 (dx + 1) + 3 (dy + 1) + (dz + 1) reads the input at
 * (x + dx, y + dy, z + dz)), the batch-norm scale [out] and shift [out];
 * then the head weight [cout][widths[0]] and bias [cout].  -1 for invalid
 * parameters.                                                               */
int64_t unet_param_count(const unet_params* p);

/* Create with seeded parameters (convolutions and head U(+-1/sqrt(fan_in)),
 * batch-norm scale 1, shift 0; running mean 0, variance 1); allocates the
 * training workspaces for max_batch.  Errors: LBM_EINVAL, LBM_ENOMEM,
 * LBM_EDEVICE.                                                             */
int unet_create(const unet_params* p, uint64_t seed, void* hip_stream, unet_net** out);

/* Copy the FP32 parameter vector in or out (host pointers); synchronises.  */
int unet_set_params(unet_net* n, const float* host_params, int64_t count);
int unet_get_params(unet_net* n, float* host_params, int64_t count);

/* Running statistics, host float [2][sum of block widths]: all running
 * means in block order, then all running variances.  Synchronises.         */
int unet_bn_stats(unet_net* n, float* host, int64_t count);

/* Forward pass: x device BF16 [B][cin][nx][ny][nz], y device FP32
 * [B][cout][nx][ny][nz].  training != 0 normalises with the batch
 * statistics and updates the running ones.  Asynchronous.                  */
int unet_forward(unet_net* n, const uint16_t* x, int32_t B, int32_t training, float* y);

/* Training-mode forward pass, masked MSE (as fno_loss_grad: mask device
 * uint8 [nx][ny][nz], target device FP32 [B][cout][nx][ny][nz]) and the
 * gradient of every parameter; host_grads (may be NULL) receives a copy,
 * *loss (may be NULL) the loss (LBM_EINVAL for an empty mask when the loss
 * is requested).  Asynchronous unless a host output is requested.          */
int unet_loss_grad(unet_net* n, const uint16_t* x, const float* target, const uint8_t* mask, int32_t B, float* loss,
                   float* host_grads);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the last gradients.   */
int unet_adam_step(unet_net* n, float lr);

/* unet_loss_grad followed by unet_adam_step.                               */
int unet_train_step(unet_net* n, const uint16_t* x, const float* target, const uint8_t* mask, int32_t B, float lr,
                    float* loss);

void unet_destroy(unet_net* n);
const char* unet_last_error(const unet_net* n);

#ifdef __cplusplus
}
#endif
#endif /* MI355LBM_H */
