/*
 * telbm.h -- C ABI of the MI355X library for the ternary free-energy entropic
 * lattice Boltzmann update of Woehrwag, Semprebon, Mazloomi, Karlin and
 * Kusumaatmaja, "Ternary free-energy entropic lattice Boltzmann model with
 * high density ratio" (arXiv:1710.07486).
 *
 * The calls follow the paper's statement of the problem: fix the free energy
 * (Eqs. 1-4), initialise the density rho, order parameter phi and velocity v
 * of Eqs. (5)-(7), advance N time steps, read the fields back.
 *
 * Conventions
 *  - Fields are arrays of doubles laid out [nz][ny][nx] with x fastest.
 *    Vector fields are three such arrays back to back (x, y, z components).
 *  - "on_device" != 0 means the pointer is a device pointer on the current
 *    HIP device; otherwise it is host memory.  The library copies; it never
 *    keeps a caller's field pointer.
 *  - Device memory: the caller allocates one arena of telbm_required_bytes()
 *    (e.g. a torch uint8 tensor) and lends it to telbm_create(); the library
 *    never allocates or frees device memory itself and never frees the arena.
 *  - Work is enqueued on the stream set by telbm_set_stream (default: the
 *    null stream).  telbm_step is asynchronous; telbm_read, telbm_diagnostics
 *    and telbm_sync synchronise that stream.
 *  - Every call returns TELBM_OK or an error code; no C++ exception crosses
 *    the ABI.  telbm_last_error gives a message for the last failed call on a
 *    handle.  Handles are not thread-safe; distinct handles are independent.
 */
#ifndef TELBM_H
#define TELBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define TELBM_OK 0
#define TELBM_ERR_INVAL 1     /* bad argument or parameter; nothing was enqueued  */
#define TELBM_ERR_UNSTABLE 2  /* non-finite value, rho <= 0 or |u_alpha| >= 1       */
#define TELBM_ERR_DEVICE 3    /* a HIP runtime call failed                          */
#define TELBM_ERR_NOMEM 4     /* arena smaller than telbm_required_bytes            */

/* Lattices: the same velocity set carries the density and the phase-field
 * populations. */
#define TELBM_D2Q9 0
#define TELBM_D3Q27 1

/* Storage precision of the populations. */
#define TELBM_FP64 0
#define TELBM_FP32_MIXED 1  /* FP32 populations: each f value is stored as its deviation
                               f_i - w_i rho_ref with rho_ref the FP64 density of the node
                               that wrote it; FP64 for the densities, the equation-of-
                               state chemical potential and the entropic stabiliser
                               ratio                                                 */

/* Fields that telbm_read can return. */
#define TELBM_FIELD_RHO 0    /* density rho                                         */
#define TELBM_FIELD_PHI 1    /* phase field phi                                     */
#define TELBM_FIELD_UX 2     /* physical velocity (j + F/2)/rho, x component        */
#define TELBM_FIELD_UY 3
#define TELBM_FIELD_UZ 4
#define TELBM_FIELD_C1 5     /* liquid-1 concentration C_l1                         */
#define TELBM_FIELD_C2 6     /* liquid-2 concentration C_l2                         */
#define TELBM_FIELD_MU_RHO 7 /* chemical potential mu_rho = dF/drho                 */
#define TELBM_FIELD_MU_PHI 8 /* chemical potential mu_phi = dF/dphi                 */
#define TELBM_FIELD_FX 9     /* thermodynamic force density, x component            */
#define TELBM_FIELD_FY 10
#define TELBM_FIELD_FZ 11

/* Liquid-gas equations of state of the bulk free energy (Eq. 2): the paper's
 * Carnahan-Starling (Eq. 4), and van der Waals and Peng-Robinson, which it
 * names as alternatives (their Psi follows from the textbook pressure through
 * p = rho Psi' - Psi, stated above Eq. 4):
 *   van der Waals  p = rho R T/(1 - b rho) - a rho^2
 *   Peng-Robinson  p = rho R T/(1 - b rho) - a alpha(T) rho^2/(1 + 2 b rho - b^2 rho^2),
 *                  alpha = [1 + m (1 - sqrt(T/T_c))]^2,
 *                  m = 0.37464 + 1.54226 omega - 0.26992 omega^2.            */
#define TELBM_EOS_CS 0
#define TELBM_EOS_VDW 1
#define TELBM_EOS_PR 2

/* Parameters (plain data, copied by telbm_create).
 *  eos                 TELBM_EOS_*; omega: acentric factor (Peng-Robinson only).
 *  a, b, R, T          constants of the equation of state (Eq. 4 for
 *                      Carnahan-Starling); T the temperature.
 *  rho_g, rho_l        coexisting gas/liquid densities; both 0 means "solve the
 *                      Maxwell construction at T" (text after Eq. 4).
 *  lambda1..3          bulk free energy weights, Eq. (2).
 *  kappa1..3           interfacial free energy weights, Eq. (3).
 *  chi                 scale of the phase field phi (definition of C_l1, C_l2).
 *  nu                  kinematic viscosity eta/rho (uniform; tau = 3 nu + 1/2).
 *  mobility            M of the Cahn-Hilliard equation (7).
 *  tau_phi             relaxation time of the phase-field populations (> 1/2).
 *  rho_ref             reserved (the FP32 form takes each writer's own density).
 *  diag_every          conservation/health diagnostics every this many steps
 *                      (0 disables).
 *  walls               1: flat solid walls at y = -1/2 and y = ny - 1/2, the
 *                      box staying periodic in x (and z) -- the wetting
 *                      boundary conditions the paper's outlook names, in the
 *                      geometric form it cites first.  Populations streaming
 *                      into a wall return with the opposite velocity (halfway
 *                      bounce-back: no slip, no flux of mass or phi).  The
 *                      stencils see one ghost row beyond each wall: for rho and
 *                      phi psi(ghost) = psi(wall row) + cot(theta) |grad_t psi|
 *                      (central differences along the wall), which imposes
 *                      n.grad psi = -cot(theta) |grad_t psi|, theta the contact
 *                      angle measured in the phase where psi is large; for the
 *                      chemical potentials the ghost repeats the wall row.
 *                      theta_* in (0, pi); pi/2 is neutral.  Needs ny >= 2
 *                      (TELBM_ERR_INVAL).
 *  glattice            lattice of the phase-field populations g, which the
 *                      paper leaves open: 0 the lattice of f; 1 its rest and
 *                      axis directions (D2Q5 / D3Q7) with axis weights 1/6 and
 *                      the equilibrium to first order in u,
 *                      g_i = (1/6)(3 Gamma mu_phi + 3 phi c_i.u), g_0 = phi - sum,
 *                      which keeps the moments phi, phi u and Gamma mu_phi I of
 *                      Eq. (7) and moves 2 (Q + 5 or 7) instead of 4 Q values
 *                      per node and step.  Not available for D3Q27 in the
 *                      FP32-mixed form nor in the batched form
 *                      (TELBM_ERR_INVAL).
 * Validation: 0 < T < T_c, rho_l > rho_g > 0, nu > 0, tau_phi > 1/2, chi != 0,
 * sizes >= 1 (nz == 1 for D2Q9), nx*ny*nz < 2^29 (the kernels address each
 * FP64 slice of N values with 32-bit byte offsets).                        */
typedef struct telbm_params {
    int32_t lattice;
    int32_t precision;
    int32_t nx, ny, nz;
    int32_t eos;              /* TELBM_EOS_*: the liquid-gas equation of state  */
    double a, b, R, T;
    double rho_g, rho_l;
    double lambda1, lambda2, lambda3;
    double kappa1, kappa2, kappa3;
    double chi;
    double nu;
    double mobility;
    double tau_phi;
    double rho_ref;
    uint32_t diag_every;
    uint32_t reserved1;
    double omega;             /* Peng-Robinson acentric factor (TELBM_EOS_PR)    */
    int32_t walls;            /* 0: periodic box; 1: solid walls normal to y     */
    uint32_t reserved2;
    double theta_rho_lo, theta_rho_hi;  /* contact angles (radians) of the walls */
    double theta_phi_lo, theta_phi_hi;  /* at y = -1/2 (lo) and ny - 1/2 (hi)    */
    int32_t glattice;         /* phase-field lattice: 0 as for f, 1 reduced      */
    uint32_t reserved3;
} telbm_params;

/* Diagnostics of the state before step `step` (the last diagnosed step):
 * totals of rho, phi and momentum j = sum_i f_i c_i; max |u_phys|; min rho;
 * min/max of the entropic stabiliser gamma of that step's collision; count
 * of nodes with a non-finite rho, phi or velocity. */
typedef struct telbm_diag {
    int64_t step;
    double mass;
    double phi_total;
    double mom[3];
    double max_u;
    double min_rho;
    double gamma_min;
    double gamma_max;
    int64_t nonfinite;
} telbm_diag;

typedef struct telbm_solver telbm_solver;

/* Version string of the library build. */
const char *telbm_version(void);

/* Critical temperature of the Carnahan-Starling EOS (dp/drho = d2p/drho2 = 0).
 * Writes T_c; returns TELBM_ERR_INVAL for a, b, R not positive. */
int telbm_critical_temperature(double a, double b, double R, double *T_c);

/* Maxwell construction at temperature T (the common tangent stated after
 * Eq. 4): coexisting densities and the constants C, Psi0 that make
 * Psi(rho_g) = Psi(rho_l) = Psi0 with Psi'(rho_g) = Psi'(rho_l) = 0.
 * Host only, stateless.  TELBM_ERR_INVAL if T is not in (0, T_c). */
int telbm_coexistence(double a, double b, double R, double T,
                      double *rho_g, double *rho_l, double *C, double *Psi0);

/* Temperature whose Maxwell ratio rho_l/rho_g equals `ratio` (> 1). */
int telbm_temperature_for_ratio(double a, double b, double R, double ratio, double *T);

/* The same three for any TELBM_EOS_* (omega used by Peng-Robinson only; its
 * T_c is that of alpha = 1).  TELBM_ERR_INVAL for an unknown eos. */
int telbm_eos_critical_temperature(int eos, double a, double b, double R, double omega, double *T_c);
int telbm_eos_coexistence(int eos, double a, double b, double R, double omega, double T,
                          double *rho_g, double *rho_l, double *C, double *Psi0);
int telbm_eos_temperature_for_ratio(int eos, double a, double b, double R, double omega, double ratio,
                                    double *T);

/* Bytes of device arena telbm_create needs for these parameters. */
int telbm_required_bytes(const telbm_params *p, size_t *bytes);

/* Create a solver.  `device_arena` (device pointer, >= required bytes, 256-byte
 * aligned) is borrowed for the solver's lifetime.  The state is undefined
 * until telbm_init_fields. */
int telbm_create(const telbm_params *p, void *device_arena, size_t bytes, telbm_solver **out);

/* Enqueue all further work of this solver on `stream` (a hipStream_t). */
int telbm_set_stream(telbm_solver *s, void *stream);

/* Initialise the populations at equilibrium with the given fields (the
 * entropic equilibrium for rho, u and the phase-field equilibrium for phi,
 * with mu_phi evaluated from rho and phi).  rho and phi are required; u may
 * be NULL for zero velocity, else 2 (D2Q9) or 3 (D3Q27) component arrays.
 * Returns TELBM_ERR_UNSTABLE (state unchanged) if any rho <= 0, any value is
 * non-finite or any |u_alpha| >= 1.  Resets the step counter. */
int telbm_init_fields(telbm_solver *s, const double *rho, const double *phi, const double *u,
                      int on_device);

/* Advance n >= 0 time steps (asynchronous).  A diagnosed unstable state is
 * reported by the next synchronising call. */
int telbm_step(telbm_solver *s, int64_t n);

/* Read one field of the current state into `out` (nx*ny*nz doubles). */
int telbm_read(telbm_solver *s, int field, double *out, int on_device);

/* Latest diagnostics (runs a diagnostic pass of the current state if none has
 * been taken since the last step).  Synchronises.  Returns TELBM_ERR_UNSTABLE
 * (with `out` filled) if the state is unstable. */
int telbm_diagnostics(telbm_solver *s, telbm_diag *out);

/* The diagnostics taken last, by a diagnosed step (diag_every) or by
 * telbm_diagnostics, without a new pass: a step's own reduction costs no
 * extra launch.  `out->step` is the step whose starting state they describe
 * (-1: none taken since telbm_init_fields).  Synchronises.  Returns
 * TELBM_ERR_UNSTABLE (with `out` filled) if that state was unstable. */
int telbm_last_diagnostics(telbm_solver *s, telbm_diag *out);

/* Wait for the solver's stream; reports pending instability. */
int telbm_sync(telbm_solver *s);

/* Steps taken since telbm_init_fields. */
int telbm_step_count(const telbm_solver *s, int64_t *steps);

/* Kernel-level timing: run n steps recording a HIP event pair around each
 * kernel launch, and return the mean duration in milliseconds of each kernel
 * kind (ms[k] for k < *kinds; names via telbm_kernel_name) and, in
 * ms[*kinds], the mean time per step over the whole span from the first
 * launch's start event to the last launch's end event.  `ms` must hold at
 * least 4 values (3 kinds + the span).  Synchronises. */
int telbm_time_kernels(telbm_solver *s, int64_t n, double *ms, int *kinds);
const char *telbm_kernel_name(const telbm_solver *s, int kind);

/* Algorithmic bytes moved per lattice update: read and write of every f and
 * g population once (2 * 2Q * bytes per population). */
double telbm_algorithmic_bytes_per_update(const telbm_solver *s);

int telbm_destroy(telbm_solver *s);
const char *telbm_last_error(const telbm_solver *s);


/* ------------------------------------------------------------------------- */
/* Batched form: many lattices of uneven size and parameters advanced        */
/* together.  All instances share lattice and precision; each has its own    */
/* sizes, temperature, free-energy and transport parameters.  Each phase of  */
/* a step is one persistent launch over a work list of (instance, tile)      */
/* items; runs of an even number of steps are replayed from captured HIP     */
/* graphs.  Members may have walls (each with its own contact angles) beside */
/* periodic ones; the reduced phase-field lattice is not available here      */
/* (TELBM_ERR_INVAL).  Diagnostics are not collected in this form.          */
/* ------------------------------------------------------------------------- */
typedef struct telbm_batch telbm_batch;

/* Arena bytes for `count` instances with parameters p[0..count-1]. */
int telbm_batch_required_bytes(const telbm_params *p, int count, size_t *bytes);

/* Create a batch in a borrowed, 256-byte aligned device arena. */
int telbm_batch_create(const telbm_params *p, int count, void *device_arena, size_t bytes,
                       telbm_batch **out);

int telbm_batch_set_stream(telbm_batch *b, void *stream);

/* Number of compiled tile shapes and the shape (threads along x, y) of one. */
int telbm_batch_tile_variants(int *count);
int telbm_batch_tile_shape(int variant, int *bx, int *by);

/* Select the tile shape and the persistent grid size (workgroups per compute
 * unit, 1..64).  Synchronises the stream and drops captured graphs. */
int telbm_batch_set_tiles(telbm_batch *b, int variant, int wg_per_cu);

/* Steps per captured graph (even; 0 disables graphs).  Default 10. */
int telbm_batch_set_graph_steps(telbm_batch *b, int steps_per_graph);

/* Step mode of a D2Q9 batch: 0 (default) the persistent launches above; 1
 * every instance takes the single solver's fused one-launch step, the
 * instances on parallel branches of the captured graphs; 2 the same fused
 * step for all instances in one launch over an (instance, 64 x 8 tile) work
 * list (one launch per equation of state present).  The fused step moves
 * 332 B/node against ~480 for the three-phase step.  The state carries over
 * between the modes; may be changed between steps.  TELBM_ERR_INVAL for
 * D3Q27 batches or other values. */
int telbm_batch_set_mode(telbm_batch *b, int mode);

/* Initialise instance idx (same semantics as telbm_init_fields).  Every
 * instance must be initialised before the first telbm_batch_step. */
int telbm_batch_init_fields(telbm_batch *b, int idx, const double *rho, const double *phi,
                            const double *u, int on_device);

/* Advance all instances n steps (asynchronous). */
int telbm_batch_step(telbm_batch *b, int64_t n);

/* Read one field of instance idx (synchronises). */
int telbm_batch_read(telbm_batch *b, int idx, int field, double *out, int on_device);

int telbm_batch_sync(telbm_batch *b);
int telbm_batch_step_count(const telbm_batch *b, int64_t *steps);
int telbm_batch_destroy(telbm_batch *b);
const char *telbm_batch_last_error(const telbm_batch *b);

/* ------------------------------------------------------------------------- */
/* Learned form: kernels of a convolutional surrogate (3x3 filters, circular  */
/* padding) on NHWC BF16 activations (uint16 storage) with FP32 accumulation */
/* on the matrix cores.  Channel counts must be 32 or 64 (fields with fewer  */
/* channels are stored zero-padded to 32).  Weights: FP32 masters            */
/* w[tap][ci][co] (tap = 3 (dy+1) + (dx+1)), packed to BF16 by               */
/* telbm_conv_pack_weights.  All pointers are device pointers; work is       */
/* enqueued on `stream`.  The training loop lives in the caller.             */
/* The paper has no learned part: these calls serve a surrogate that maps a  */
/* state (the density and the two liquid concentrations of Sec. 2) to the   */
/* state a fixed number of steps later.  Errors: TELBM_ERR_INVAL for a NULL  */
/* required pointer, a non-positive size or an unsupported channel count;   */
/* TELBM_ERR_NOMEM for a missing or short workspace; TELBM_ERR_DEVICE when a */
/* launch fails.  Buffers are owned by the caller; nothing is allocated.     */
/* ------------------------------------------------------------------------- */

/* Pack w (FP32, 9*cin*cout) into the forward layout wf[co][tap*cin + ci] and
 * the data-gradient layout wd[ci][tap*cout + co] with taps flipped (BF16). */
int telbm_conv_pack_weights(const float *w, int cin, int cout, void *wf_bf16, void *wd_bf16, void *stream);

/* y[p][co] = act(bias[co] + sum_{tap,ci} x[p + d off(tap)][ci] w[tap][ci][co])
 * over an n x h x w periodic grid, off(tap) = (tap/3 - 1, tap%3 - 1) in
 * (row, column), dilation d = `dilation` >= 1; act = ReLU if relu != 0.
 * bias may be NULL.  Writes y_bf16 and/or y_f32 (either may be NULL, not
 * both). */
int telbm_conv_forward(const void *x, int n, int h, int w, int cin, const void *wf_bf16, const float *bias,
                       int cout, int dilation, int relu, void *y_bf16, float *y_f32, void *stream);

/* Gradients of the linear part of telbm_conv_forward given dy (BF16,
 * n*h*w*cout): dx (BF16, optional) = sum_t dy[p - d off(t)] w[t]^T,
 * multiplied by (x_relu_mask > 0) when a mask (the ReLU output that fed
 * this layer) is given; dw (FP32, optional) = sum_p x[p + d off(t)] dy[p]^T;
 * db (FP32, optional) = sum_p dy[p].  dw and db need a workspace of
 * telbm_conv_workspace_bytes; the reductions are deterministic. */
int telbm_conv_backward(const void *x, const void *dy, int n, int h, int w, int cin, int cout, int dilation,
                        const void *wd_bf16, const void *x_relu_mask, void *dx_bf16, float *dw, float *db,
                        void *workspace, size_t workspace_bytes, void *stream);
int telbm_conv_workspace_bytes(int n, int h, int w, int cin, int cout, size_t *bytes);

/* Residual head and loss over `pixels` x `channels` (first `valid` used):
 * pred = x + y; with a target, dy = 2 (pred - target)/(pixels*valid) (BF16)
 * and per-block partial sums of (pred - target)^2 into loss_partials
 * (*nblocks of them).  pred (FP32) is optional. */
int telbm_residual_mse(const void *x, const float *y, const void *target, int64_t pixels, int channels,
                       int valid, void *dy_bf16, float *pred, float *loss_partials, int *nblocks, void *stream);

/* Network input from a state (FP64 rho, phi and optionally the velocity
 * ux, uy; `pixels` values each): BF16 NHWC with 32 channels, channel 0 =
 * (rho - rho_g)/(rho_l - rho_g), channel 1 = C1 = (ch0 + phi/chi)/2,
 * channel 2 = C2 = (ch0 - phi/chi)/2 (the concentrations of Sec. 2 with
 * C_g = 1 - ch0), channels 3, 4 = u_scale ux, u_scale uy (zero when ux or uy
 * is NULL), channels 5..31 zero. */
int telbm_surrogate_encode(const double *rho, const double *phi, const double *ux, const double *uy,
                           int64_t pixels, double rho_g, double rho_l, double chi, double u_scale, void *x_bf16,
                           void *stream);

/* State from the network output y (FP32 NHWC, 32 channels, first five
 * used) and the exact input state (n images of h x w; ux_in, uy_in may be
 * NULL for a state at rest): the encoded input plus y (residual head),
 * clamped to rho >= rho_g/2 and |phi| <= 1.1 chi, then projected so that each
 * image's totals of rho, phi and rho u equal the input's (the quantities
 * the method conserves): the rho and phi defects are added in proportion to
 * w = |grad ch0| + |grad(phi/chi)| + 1e-6, the momentum defect by a uniform
 * velocity shift.  Writes rho, phi, ux, uy (FP64, n*h*w each); needs
 * telbm_surrogate_decode_workspace_bytes of workspace. */
int telbm_surrogate_decode(const float *y, const double *rho_in, const double *phi_in, const double *ux_in,
                           const double *uy_in, int n, int h, int w, double rho_g, double rho_l, double chi,
                           double u_scale, double *rho_out, double *phi_out, double *ux_out, double *uy_out,
                           void *workspace, size_t workspace_bytes, void *stream);
int telbm_surrogate_decode_workspace_bytes(int n, int h, int w, size_t *bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * decode as telbm_surrogate_decode, with its workspace in a static device
 * array of telbm_surrogate_decode_noalloc_max_bytes() = 16 MiB that the
 * library holds on each GPU it runs on until the process ends.  Calls no
 * hipMalloc, hipFree or allocating routine.  Returns TELBM_ERR_NOMEM when the
 * decode needs more workspace than that (telbm_surrogate_decode_workspace_bytes;
 * about 2 million pixels), TELBM_ERR_INVAL for invalid arguments as
 * telbm_surrogate_decode, TELBM_ERR_DEVICE if the array's address cannot be
 * obtained on the current device.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (on different streams, or from
 * different threads) race and must be serialised by the caller. */
int telbm_surrogate_decode_noalloc(const float *y, const double *rho_in, const double *phi_in, const double *ux_in,
                                   const double *uy_in, int n, int h, int w, double rho_g, double rho_l, double chi,
                                   double u_scale, double *rho_out, double *phi_out, double *ux_out, double *uy_out,
                                   void *stream);
size_t telbm_surrogate_decode_noalloc_max_bytes(void);

/* ------------------------------------------------------------------------- */
/* Three liquids and the gas: the extension to more liquid components named   */
/* in the paper's concluding paragraph (one more double well in the bulk      */
/* energy of Eq. 2 and one more gradient term in Eq. 3 per added liquid).     */
/* A second phase field psi carries liquid 3:                                 */
/*   C1 = (C_L + phi/chi - psi/chi)/2, C2 = (C_L - phi/chi - psi/chi)/2,      */
/*   C3 = psi/chi, C_L = 1 - C_g (C_g as defined below Fig. 1),              */
/* so psi = 0 is the paper's two-liquid model; the pure phases are           */
/* (rho_g, 0, 0), (rho_l, chi, 0), (rho_l, -chi, 0), (rho_l, 0, chi).          */
/* f_B gains (lambda4/2) C3^2 (1-C3)^2, f_I gains (kappa4/2) |grad C3|^2.     */
/* The potentials are the chain rule through C_m: with                       */
/* nu_m = lambda_{m+1} W(C_m) - kappa_{m+1} lap C_m, W(C) = C(1-C)(1-2C),     */
/*   mu_rho = (lambda1/2) Psi' - kappa1 lap rho - (nu1 + nu2)/(2 (rho_g - rho_l)), */
/*   mu_phi = (nu1 - nu2)/(2 chi), mu_psi = (2 nu3 - nu1 - nu2)/(2 chi).      */
/* The force gains -psi grad mu_psi; phi and psi follow Cahn-Hilliard         */
/* equations (Eq. 7) with the mobility matrix M m of telbm_nl_mobility,       */
/* realised by two phase-field BGK populations whose equilibria take the     */
/* mixed potentials (m mu)_phi and (m mu)_psi.  FP64, periodic boxes, the    */
/* phase fields on the lattice of f; walls, the FP32-mixed form, the reduced */
/* phase-field lattice and the batched form reject it (TELBM_ERR_INVAL).     */
/* ------------------------------------------------------------------------- */
typedef struct telbm_nl_params {
    double lambda4, kappa4; /* double well and gradient coefficient of liquid 3 (kappa4 > 0) */
} telbm_nl_params;

typedef struct telbm_nl telbm_nl;

#define TELBM_NL_FIELD_RHO 0
#define TELBM_NL_FIELD_PHI 1
#define TELBM_NL_FIELD_PSI 2
#define TELBM_NL_FIELD_UX 3      /* physical velocity (j + F/2)/rho */
#define TELBM_NL_FIELD_UY 4
#define TELBM_NL_FIELD_UZ 5
#define TELBM_NL_FIELD_C1 6      /* concentrations of the three liquids */
#define TELBM_NL_FIELD_C2 7
#define TELBM_NL_FIELD_C3 8
#define TELBM_NL_FIELD_MU_RHO 9
#define TELBM_NL_FIELD_MU_PHI 10
#define TELBM_NL_FIELD_MU_PSI 11
#define TELBM_NL_FIELD_FX 12     /* thermodynamic force density */
#define TELBM_NL_FIELD_FY 13
#define TELBM_NL_FIELD_FZ 14

/* The (phi, psi) mobility matrix divided by M, as {pp, ps, sp, ss}: the image
 * under the map above of the concentration mobility of consistent N-phase
 * Cahn-Hilliard models (Boyer and Lapuerta) with inverse phase weights
 * w = (1/kappa2, 1/kappa3, 1/kappa4), W = w1 + w2 + w3,
 *   M_C = (M / chi^2) (diag(w) - w w^T / W) / (w1 + w2),
 * which is, in closed form,
 *   pp = (4 w1 w2 + (w1 + w2) w3) / (W (w1 + w2)),
 *   ps = sp = w3 (w2 - w1) / (W (w1 + w2)),  ss = w3 / W.
 * At an interface between two liquids where the third is absent it sends the
 * absent liquid's diffusive flux to zero when lambda_m / kappa_m is the same
 * for all liquids.  For kappa2 = kappa3, pp = 1 and ps = 0: phi moves exactly
 * as in the two-liquid model (diag(1, 1/3) for equal kappas).  Host only;
 * TELBM_ERR_INVAL unless kappa2, kappa3, kappa4 > 0. */
int telbm_nl_mobility(const telbm_params *p, const telbm_nl_params *q, double *m);

/* Bytes of device arena for these parameters (two population buffers of
 * 3 Q N doubles, six N-double fields and, for D3Q27, the partial next-step
 * moments of the z-column collision, (rho, phi) pairs and psi, with their
 * tile inboxes; each part 256-byte aligned). */
int telbm_nl_required_bytes(const telbm_params *p, const telbm_nl_params *q, size_t *bytes);

/* Create, borrowing `device_arena` (>= required bytes, 256-byte aligned) for
 * the solver's lifetime.  Parameters as for telbm_create plus q;
 * p->precision must be TELBM_FP64, p->walls and p->glattice 0. */
int telbm_nl_create(const telbm_params *p, const telbm_nl_params *q, void *device_arena, size_t bytes,
                    telbm_nl **out);
int telbm_nl_set_stream(telbm_nl *s, void *stream);

/* Equilibrium populations of rho, phi, psi (required) and u (NULL: at rest;
 * else D component arrays), the phase-field equilibria with the mixed
 * potentials of those fields.  TELBM_ERR_UNSTABLE (state unchanged) if any
 * rho <= 0, any value is non-finite or any |u_alpha| >= 1.  Resets the step
 * counter. */
int telbm_nl_init_fields(telbm_nl *s, const double *rho, const double *phi, const double *psi, const double *u,
                         int on_device);

/* Advance n >= 0 time steps (asynchronous): moments, potentials, collision.
 * On D3Q27 the collision also leaves the next step's moments as partial sums,
 * which the next step (or a read) completes in the same pass that computes the
 * potentials, instead of a pass over the populations. */
int telbm_nl_step(telbm_nl *s, int64_t n);

/* One TELBM_NL_FIELD_* of the current state into `out` (N doubles). Synchronises. */
int telbm_nl_read(telbm_nl *s, int field, double *out, int on_device);
int telbm_nl_step_count(const telbm_nl *s, int64_t *steps);
int telbm_nl_destroy(telbm_nl *s);
const char *telbm_nl_last_error(const telbm_nl *s);

/* One Adam step (Kingma and Ba 2015) on n FP32 weights at step t >= 1. */
int telbm_adam_step(float *w, const float *g, float *m, float *v, int64_t n, float lr, float beta1,
                    float beta2, float eps, int64_t t, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TELBM_H */
