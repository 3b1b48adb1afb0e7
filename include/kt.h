/*
 * kt.h -- C ABI of the MI355X Kurganov-Tadmor step library.
 *
 * One Kurganov-Tadmor (KT) semi-discrete step with Heun (two-stage SSP
 * Runge-Kutta) time integration of (3+1)d second-order viscous hydrodynamics
 * in Milne coordinates (tau, x, y, eta_s), for T^{tau mu}, the shear stress
 * pi^{mu nu} and the bulk pressure Pi, with per-cell recovery of the energy
 * density e and the flow u^mu.  Bazow, Heinz & Strickland, arXiv:1608.06577:
 * equations of motion in Sec. 2.4 and App. B, numerical scheme in Sec. 3.1,
 * regulator in Sec. 3.2, lattice and boundary conditions in Sec. 4.1, program
 * flow of one time step in Sec. 4.3.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units: fm-based natural units; e, p in fm^-4, T in fm^-1, tau in fm/c,
 *        x, y in fm, eta_s dimensionless.
 * Layout: every field is a separate device array (structure of arrays) over
 *        the physical cells only, nx*ny*neta doubles, x fastest and eta_s
 *        slowest: cell (i, j, k) is element (k*ny + j)*nx + i.  Ghost cells
 *        are not stored: the boundary conditions of Sec. 4.1 (copy of the
 *        outermost layer) or periodic wrap are applied by index.
 * Components of the evolved vector q (Sec. 3.1, Eq. qComponents), in order:
 *        0..3   T^{tau tau}, T^{tau x}, T^{tau y}, T^{tau eta}
 *        4..13  pi^{tau tau}, pi^{tau x}, pi^{tau y}, pi^{tau eta}, pi^{xx},
 *               pi^{xy}, pi^{x eta}, pi^{yy}, pi^{y eta}, pi^{eta eta}
 *        14     Pi
 *        u^mu is contravariant: (u^tau, u^x, u^y, u^eta), u^eta in fm^-1.
 * Ownership: the caller owns every device buffer (workspace, inputs,
 *        outputs) and every host array; the library keeps pointers into the
 *        workspace only, which must outlive the context.
 * Streams: all device work is ordered on the stream given to kt_init.
 *        kt_init and kt_observables synchronise that stream; nothing else
 *        blocks.
 * Errors: every call returns a kt_status and never aborts.  Argument errors
 *        are detected before any device work.  Device faults surface as
 *        KT_E_HIP at the next synchronising call.  kt_last_error(ctx)
 *        (kt_last_error(NULL) for failures without a context) gives a
 *        message.  Numerical events (Newton fallbacks, velocity clamps, cells
 *        at the energy floor, non-finite values) are counts in kt_obs, not
 *        errors.  A context is not thread safe.
 */
#ifndef KT_H
#define KT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kt_ctx kt_ctx;

typedef enum {
    KT_OK = 0,
    KT_E_ARG = 1,          /* invalid argument */
    KT_E_ALLOC = 2,        /* workspace too small */
    KT_E_HIP = 3,          /* HIP runtime or device error */
    KT_E_STATE = 4,        /* call not valid in the context's state */
    KT_E_UNSUPPORTED = 5   /* valid request the library does not implement */
} kt_status;

enum { KT_FP64 = 0, KT_MIXED = 1 };           /* kt_params.precision */
enum { KT_MILNE = 0, KT_CARTESIAN = 1 };       /* Cartesian: metric diag(1,-1,-1,-1), no geometric sources (Sec. 5.1) */
enum { KT_BC_OUTFLOW = 0, KT_BC_PERIODIC = 1 };
enum { KT_ZETA_LINEAR = 0, KT_ZETA_PAPER = 1 }; /* kt_params.zeta_model */

/* Equation of state (Sec. 2.3).  conformal != 0: p = e/3, c_s^2 = 1/3,
 * T = (e/a_sb)^{1/4}.  Otherwise a table on n >= 2 ln-uniform nodes
 * e_i = exp(ln_e0 + i*dln_e) with p_i, cs2_i, T_i (host arrays, read during
 * kt_init only).  Between nodes p/e, T/e^{1/4} and c_s^2 are interpolated
 * linearly in ln e; outside the table the end node's p/e, T/e^{1/4}, c_s^2
 * are kept. */
typedef struct {
    int32_t conformal;
    double a_sb;
    int32_t n;
    double ln_e0, dln_e;
    const double *p, *cs2, *T;
} kt_eos;

/* Grid, time step and physics of one event. */
typedef struct {
    int32_t nx, ny, neta;          /* physical cells, each >= 1 */
    double dx, dy, deta;           /* cell sizes, > 0 */
    double tau0, dtau;             /* initial time and step, > 0 */
    int32_t coords;                /* KT_MILNE or KT_CARTESIAN */
    int32_t bc[3];                 /* per axis x, y, eta: KT_BC_OUTFLOW or KT_BC_PERIODIC */
    double theta;                  /* generalized minmod parameter in [1, 2] (Sec. 3.1) */
    double eta_over_s;             /* eta/s >= 0; 0 = ideal, pi not evolved */
    double zeta_coef;              /* >= 0; 0 = Pi not evolved.  KT_ZETA_LINEAR: zeta/s =
                                    * zeta_coef (1/3 - c_s^2); KT_ZETA_PAPER: zeta_coef is the
                                    * normalisation of the zeta/s(T) of Sec. 2.2 (Eq. zetas) */
    double taupipi;                /* tau_pipi / tau_pi (10/7 near the conformal limit, Sec. 2.2) */
    int32_t regulate;              /* apply the regulator of Sec. 3.2 */
    int32_t regulate_bulk;         /* the regulator factor also rescales Pi */
    double xi0, rho_max;           /* regulator constants (0.1 and 1 in Sec. 3.2) */
    double e_floor;                /* energy-density floor, > 0 */
    double m2_delta;               /* velocity clamp margin of the inversion, in (0, 1) */
    int32_t floor_resets_q;        /* a cell put on the floor gets q = (e_floor,0,0,0; 0; 0) */
    double newton_tol;             /* stop when |f(e)| <= newton_tol * E, then one more step */
    int32_t newton_max;            /* Newton iterations before the bisection fallback */
    int32_t precision;             /* KT_FP64, or KT_MIXED: T^{tau mu} stored and accumulated in
                                    * FP64; pi, Pi, e, p, u and face speeds stored in FP32, flux
                                    * and source arithmetic in FP32, inversion and regulator in
                                    * FP64 */
    int32_t zeta_model;            /* KT_ZETA_LINEAR or KT_ZETA_PAPER.  In both, zeta/tau_Pi =
                                    * 15 (1/3 - c_s^2)^2 (e + P) (Sec. 2.2), so 1/tau_Pi =
                                    * 15 (1/3 - c_s^2)^2 T / (zeta/s) */
    double zeta_tc;                /* T_c of KT_ZETA_PAPER (> 0), in the EOS's temperature unit;
                                    * ignored by KT_ZETA_LINEAR */
    int32_t reduced;               /* 0, or 1: reduced state (Sec. 2.4 and Sec. 4.2).  The step
                                    * evolves T^{tau mu}, pi^{xx}, pi^{xy}, pi^{x eta}, pi^{yy},
                                    * pi^{y eta} and Pi; pi^{tau mu} and pi^{eta eta} follow from
                                    * u_mu pi^{mu nu} = 0 and pi^mu_mu = 0 (Eqs. pi_tautau ..
                                    * pi_etaeta).  Each recovery solves for (e, u) and those five
                                    * together (a fixed point over u, started from the flow before
                                    * the stage, to 1e-14 u^tau, at most 100 passes) and stores
                                    * them beside the five, so the face and source kernels read the
                                    * whole tensor; the flux and stage updates skip them.  The
                                    * initial state's pi^{tau mu} and pi^{eta eta} are not read.
                                    * Newton starts from the conformal closed form only
                                    * (kt_set_inv_start: KT_E_UNSUPPORTED for another start). */
} kt_params;

/* Initial data on the device, in one of three forms:
 *   - q[0..14] (conserved form; all 15 non-null), e null: (e, u) are
 *     recovered from q (Sec. 2.4);
 *   - the primitives e, u[4], pi[10] and Pi (all non-null), q null: the library
 *     forms T^{tau mu} with Eqs. Ttt, Tti of Sec. 2.4, then recovers (e, u);
 *   - resume: q[0..14], e and u[4] (all non-null), as kt_observables exports
 *     them (kt_fields), taken as they are, with p (nullable; p(e) of the EOS
 *     when null) and u_prev: no recovery runs, so a run continued from an
 *     exported state (q, e, p, u, u_prev at the exported tau as tau0) is bit
 *     for bit the uninterrupted one.
 * u_prev (nullable) is the previous-step flow; when null u^{-1} = u^0
 * (Sec. 4.3).  pi and Pi are not read in the other two forms. */
typedef struct {
    const double *q[15];
    const double *e;
    const double *u[4];
    const double *pi[10];
    const double *Pi;
    const double *u_prev[4];
    const double *p;
} kt_init_state;

/* Device destinations for kt_observables; every entry may be null.  p is the
 * equilibrium pressure p(e) the step uses. */
typedef struct {
    double *e;
    double *u[4];
    double *q[15];
    double *u_prev[4];
    double *p;
} kt_fields;

/* Diagnostics of the current state (all reductions are deterministic). */
typedef struct {
    double tau;
    int64_t step;
    double energy;                 /* sum T^{tau tau} * (tau) dx dy deta  (tau only in Milne) */
    double momentum[3];            /* same for T^{tau x}, T^{tau y}, T^{tau eta} */
    double e_max, T_max;
    double v_max;                  /* max over cells and axes of |u^i / u^tau| (eta: times tau) */
    double cfl;                    /* dtau * max_i |v^i| / d_i */
    double norm_err;               /* max |u.u - 1| */
    double pi_transverse;          /* max |pi^{mu nu} u_nu| / sqrt(pi:pi) (tetrad components) */
    double pi_trace;               /* max |pi^mu_mu| / sqrt(pi:pi) */
    int64_t n_nan;                 /* cells with a non-finite value in q, e or u */
    /* recovery counters accumulated since kt_init */
    int64_t newton_iters_cells, n_recover_cells;
    int64_t newton_iters_faces, n_recover_faces;
    int64_t n_floor, n_clamp, n_fallback;   /* cells */
    int64_t n_fallback_faces;               /* face states solved by bisection */
    /* reduced state (kt_params.reduced): passes of the recoveries' fixed point
     * (each one inversion; newton_iters_cells sums the iterations of every
     * pass) and cell recoveries that reached the pass limit without meeting
     * the tolerance; 0 otherwise */
    int64_t fp_passes, fp_not_converged;
} kt_obs;

/* Device workspace needed for p and eos (bytes, multiple of 256), 0 if the
 * arguments are invalid. */
size_t kt_workspace_bytes(const kt_params *p, const kt_eos *eos);

/* Create a context: copy the EOS into the workspace, form q^0 (from
 * primitives if given), recover (e^0, u^0) at tau0 (Sec. 2.4, Eqs. eInferred,
 * utInferred, uiInferred), set u^{-1}.  d_ws: device memory of ws_bytes >=
 * kt_workspace_bytes(p, eos), 256-byte aligned.  Synchronises stream.
 * Errors: KT_E_ARG (sizes, spacings, theta outside [1,2], tau0 <= 0 in
 * Milne, dtau <= 0, e_floor <= 0, table with n < 2, null pointers),
 * KT_E_ALLOC (workspace too small), KT_E_HIP. */
kt_status kt_init(const kt_params *p, const kt_eos *eos, const kt_init_state *s0,
                  void *d_ws, size_t ws_bytes, hipStream_t stream, kt_ctx **out);

/* kt_init without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, serving loops, harnesses that
 * forbid hipMalloc): the context's workspace is the library's own static
 * device array of KT_STATIC_WS_BYTES bytes, one per GPU, set up with the
 * library's code object and held until the process ends.  Neither this call
 * nor any later call on the context allocates device memory (the context
 * itself lives on the host heap, as for kt_init).  Every context made this
 * way on one GPU shares that GPU's array: a new one overwrites the state of
 * the previous one on the same device, which must not be used afterwards,
 * and contexts whose calls overlap on one GPU race.  The state is set up as
 * by kt_init (nothing is assumed about the array's previous contents).
 * Errors: those of kt_init; KT_E_ALLOC when kt_workspace_bytes(p, eos)
 * exceeds KT_STATIC_WS_BYTES; KT_E_HIP when the array's device address
 * cannot be obtained on the current device.  Release with kt_destroy. */
#define KT_STATIC_WS_BYTES (64u << 20)
kt_status kt_init_static(const kt_params *p, const kt_eos *eos, const kt_init_state *s0,
                         hipStream_t stream, kt_ctx **out);

/* Enqueue n_steps >= 0 full Heun steps (Sec. 3.1, Eqs. step1-finalStep with
 * s = 2; order of Sec. 4.3): stage 1 at tau^n, recovery and regulation of q*
 * and stage 2 at tau^{n+1}, Heun average, recovery and regulation of
 * q^{n+1}.  Asynchronous. */
kt_status kt_step(kt_ctx *c, int32_t n_steps);

/* Standalone inversion of n cells at time tau (Sec. 2.4 and Sec. 3.2):
 * in[0..8] = device arrays T^{tau tau}, T^{tau x}, T^{tau y}, T^{tau eta},
 * pi^{tau tau}, pi^{tau x}, pi^{tau y}, pi^{tau eta}, Pi (Pi may be null = 0).
 * Outputs e_out[n], u_out[4][n]; iters_out and flags_out (bit 1 floor,
 * 2 clamp, 4 bisection fallback) may be null.  Uses the context's EOS and
 * guards; Newton starts from the conformal closed form, or from the network
 * when the context's start is KT_START_LEARNED.  Asynchronous. */
kt_status kt_recover(kt_ctx *c, int64_t n, double tau, const double *const in[9],
                     double *e_out, double *const u_out[4], int32_t *iters_out,
                     int32_t *flags_out);

/* Standalone coupled recovery of n reduced states at time tau (Sec. 2.4; the
 * recovery of a kt_params.reduced step without its regulator and floor
 * reset): in[0..9] = device arrays T^{tau tau}, T^{tau x}, T^{tau y},
 * T^{tau eta}, pi^{xx}, pi^{xy}, pi^{x eta}, pi^{yy}, pi^{y eta}, Pi (Pi may be
 * null = 0).  pi^{tau mu} and pi^{eta eta} follow from u_mu pi^{mu nu} = 0 and
 * pi^mu_mu = 0 with the flow, so (e, u) and they are solved together: a fixed
 * point over u started at rest, each pass one inversion (the first from the
 * conformal closed form, later ones from the previous pass's e), stopped when
 * no component of u moves by more than 1e-14 u^tau (the eta component times
 * sqrt(g33)), on the floor state, without shear (eta_over_s = 0: one pass), or
 * after 100 passes.  Outputs e_out[n], u_out[4][n]; pi_out (nullable; else
 * five non-null arrays) receives pi^{tau tau}, pi^{tau x}, pi^{tau y},
 * pi^{tau eta}, pi^{eta eta} of the final flow; passes_out (nullable) the
 * passes, negative when the limit ended them; flags_out (nullable) the last
 * inversion's flags (bit 1 floor, 2 clamp, 4 bisection fallback).  Uses the
 * context's EOS, guards and transport switches whatever its kt_params.reduced.
 * KT_E_ARG for n < 0, null required arrays or tau <= 0 in Milne coordinates.
 * Asynchronous. */
kt_status kt_recover_reduced(kt_ctx *c, int64_t n, double tau, const double *const in[10],
                             double *e_out, double *const u_out[4], double *const pi_out[5],
                             int32_t *passes_out, int32_t *flags_out);

/* ---------------------------------------------------------------------
 * Learned start of the cell inversion.  Newton's method (Sec. 3.2) needs a
 * starting e; the paper leaves it open.  A network 11 -> 64 -> 64 -> 4 with
 * GELU(a) = a Phi(a) maps features of one state to (e/e_c, v^x, v^y,
 * sqrt(g33) v^eta), where e_c = sqrt(4E^2 - 3M^2) - E (at least e_floor) is
 * the root for the conformal EOS without bulk, E = T^{tau tau} -
 * pi^{tau tau}, M^i = T^{tau i} - pi^{tau i}, M^2 = M_x^2 + M_y^2 +
 * g33 M_eta^2.  The start is y_0 e_c; Newton then converges to the same
 * tolerance as from any other start, with bisection as the fallback.
 * Features of a state with T0 = T^{tau tau}: T^{tau x}/T0, T^{tau y}/T0,
 * sqrt(g33) T^{tau eta}/T0, pi^{tau tau}/T0, pi^{tau x}/T0, pi^{tau y}/T0,
 * sqrt(g33) pi^{tau eta}/T0, Pi/T0, 0.1 ln T0, c_s^2(T0), p(T0)/T0
 * (g33 = tau^2 in Milne coordinates, 1 in Cartesian ones).
 *
 * Parameters: KT_MLP_NPARAMS floats W1 (64x11), b1 (64), W2 (64x64), b2,
 * W3 (4x64), b3 (4), weights row major (a = W h + b), held in the
 * context's workspace together with Adam's moments.  Batched device arrays
 * are FP32 and feature-major: x[f*n + i] (11 rows), y, targets and dy
 * [o*n + i] (4 rows), act[k*n + i] (128 rows: the pre-activations of the
 * two hidden layers).  All calls are asynchronous on the context's stream.
 * --------------------------------------------------------------------- */
enum { KT_START_WARM = 0, KT_START_CONFORMAL = 1, KT_START_LEARNED = 2 };
#define KT_MLP_NPARAMS 5188

/* Newton start of the cell recoveries in kt_step: KT_START_WARM (the cell's
 * e before the stage), KT_START_CONFORMAL (closed form of the conformal EOS;
 * the default) or KT_START_LEARNED (needs kt_mlp_set first: KT_E_STATE
 * otherwise).  kt_recover uses the network for KT_START_LEARNED and the
 * conformal closed form otherwise.  Face states always start from the
 * conformal closed form of their own state. */
kt_status kt_set_inv_start(kt_ctx *c, int32_t start);

/* Copy KT_MLP_NPARAMS parameters from d_params (device) into the context
 * and zero the Adam moments; kt_mlp_get copies them out. */
kt_status kt_mlp_set(kt_ctx *c, const float *d_params, int32_t n_params);
kt_status kt_mlp_get(kt_ctx *c, float *d_params, int32_t n_params);

/* Features x (11 x n) of n states given like kt_recover's in[9] at tau; if
 * y is non-null, also the targets (e/e_c, v^x, v^y, sqrt(g33) v^eta) from
 * the recovered e_in[n] and u_in[4][n] (then both are required). */
kt_status kt_mlp_features(kt_ctx *c, int64_t n, double tau, const double *const in[9],
                          const double *e_in, const double *const u_in[4], float *x, float *y);

/* Forward pass of n samples: y (4 x n); act (128 x n, nullable) keeps the
 * pre-activations for kt_mlp_bwd. */
kt_status kt_mlp_fwd(kt_ctx *c, int64_t n, const float *x, float *y, float *act);

/* The start factor y_0 (the network's first output) of n feature vectors x
 * (11 x n, as for kt_mlp_fwd) computed as the recoveries compute it for
 * KT_START_LEARNED: on the matrix cores, with the features, W1, W2 and the
 * first hidden layer's activations rounded to FP16, FP32 accumulation, FP32
 * biases and output layer, GELU through an erf approximation of absolute
 * error below 1.5e-7 (Abramowitz & Stegun 7.1.26).  y0[n] (device, FP32).
 * KT_E_STATE before kt_mlp_set. */
kt_status kt_mlp_y0(kt_ctx *c, int64_t n, const float *x, float *y0);

/* Weighted mean squared error over the 4 x n outputs,
 * L = sum_{o,i} w_o (y - t)^2 / (4 n) with w (host array of 4, nullable =
 * all 1, each >= 0): dy = 2 w_o (y - t) / (4 n) (nullable) and L into *loss
 * (device double, nullable). */
kt_status kt_mlp_loss(kt_ctx *c, int64_t n, const float *y, const float *t, const float *w,
                      float *dy, double *loss);

/* Gradient of sum_i <dy_i, y_i> with respect to the parameters into
 * grad[KT_MLP_NPARAMS] (overwritten).  The sum over samples is taken per
 * block and then over blocks in a fixed order, so the result does not
 * depend on scheduling. */
kt_status kt_mlp_bwd(kt_ctx *c, int64_t n, const float *x, const float *act, const float *dy,
                     float *grad);

/* One Adam step (Kingma & Ba, arXiv:1412.6980) of the context's parameters
 * with step number t >= 1. */
kt_status kt_mlp_adam(kt_ctx *c, const float *grad, float lr, float b1, float b2, float eps,
                      int32_t t);

/* Diagnostics into *host_out (nullable) and, if dev_out is non-null, copies
 * of the current fields into the given device arrays.  Synchronises. */
kt_status kt_observables(kt_ctx *c, kt_obs *host_out, const kt_fields *dev_out);

/* Validity of the effective theory (Sec. 7) on the current state, per cell
 * into caller-owned device arrays of nx*ny*neta doubles (x fastest, eta
 * slowest; each nullable): the temperature T(e); the inverse Reynolds numbers
 * of Eq. inverseReynoldsNumbers, sqrt(pi^{mu nu} pi_{mu nu}) / P(e) and
 * |Pi| / P(e), P the equilibrium pressure of the EOS; the Knudsen numbers
 * tau_pi theta and tau_Pi theta (signed; 0 where pi or Pi is not evolved),
 * theta = d_mu u^mu + u^tau/tau (Milne) from a backward difference in tau
 * against the previous step's u and central differences in x, y, eta; the
 * second-order inverse Reynolds numbers of Eq. inverseReynoldsNumbers2,
 * sqrt(J^{mu nu} J_{mu nu}) / (2 eta sqrt(sigma^{mu nu} sigma_{mu nu})) and
 * |J| / (zeta |theta|), with J^{mu nu} = 2 tau_pi pi_l^<mu omega^nu>l -
 * delta_pipi pi^{mu nu} theta - tau_pipi pi^{l<mu} sigma^{nu>}_l +
 * lambda_piPi Pi sigma^{mu nu} and J = -delta_PiPi Pi theta + lambda_Pipi
 * pi^{mu nu} sigma_{mu nu} (Eq. 14_moment_terms without particle diffusion,
 * coefficients of Sec. 2.2; 0 where the quantity is not evolved or J
 * vanishes, +inf where only the denominator does), from the full velocity
 * gradient of the same differences; and the regulation factor tanh(rho)/rho
 * of Sec. 3.2 (Eqs. regPimunu, rho) evaluated on the current state (1 where
 * the regulator is off).  Asynchronous on the context's stream; KT_E_HIP if
 * a launch fails. */
kt_status kt_validity(kt_ctx *c, double *T_out, double *rinv_pi, double *rinv_Pi, double *kn_pi,
                      double *kn_Pi, double *rinv2_pi, double *rinv2_Pi, double *reg_factor);

/* Runs Heun steps until the hottest cell is below T_f (the freeze-out
 * temperature, 155 MeV in Sec. 7, in the EOS's temperature unit) or
 * max_steps steps are done, checking kt_obs.T_max every check_every steps
 * (and before the first).  *steps_done receives the steps taken (0 if the
 * state is already below T_f).  KT_E_ARG for T_f <= 0, max_steps < 0,
 * check_every < 1 or a null steps_done; errors of kt_step and
 * kt_observables are passed on.  Synchronises at every check. */
kt_status kt_run_to_freezeout(kt_ctx *c, double T_f, int32_t max_steps, int32_t check_every,
                              int32_t *steps_done);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * the launches of kt_step.  Kernel classes: 0 = KT flux divergence and
 * stage update, 1 = cell recovery and regulator, 2 = inversion of the
 * reconstructed states at every face, 3 = source terms J of a stage.
 * kt_profile_enable(c, mask) times the launches of the classes whose bit is
 * set in mask (KT_PROFILE_ALL: every class; 0 stops; a mask outside 0..15
 * is KT_E_ARG).  Events are pooled, created on first use; each timed launch
 * adds two event records to the stream.  kt_profile_read synchronises the
 * stream, returns the totals since the last read and resets them. */
#define KT_PROFILE_ALL 15
typedef struct {
    double ms[4];                  /* summed launch durations per class */
    int64_t launches[4];
} kt_profile;

kt_status kt_profile_enable(kt_ctx *c, int32_t mask);
kt_status kt_profile_read(kt_ctx *c, kt_profile *out);

/* ---------------------------------------------------------------------
 * Batches of events.  n_events events (each its own grid and initial state;
 * the same coordinates, precision, reduced flag, tau0 and dtau) are advanced together:
 * every kernel of a Heun step is one launch over the tiles of all events,
 * and one step is captured once as a hipGraph and replayed.  Results equal
 * those of separate contexts bit for bit.  Newton starts from the
 * conformal closed form, the default start of a context.
 *
 * Workspace: kt_batch_workspace_bytes(p, n, eos) bytes (256-byte aligned,
 * caller-owned, must outlive the batch), holding every event's workspace,
 * the batch time and the per-event launch tables.  p and s0 are arrays of
 * n_events entries; kt_batch_init synchronises the stream.
 * kt_batch_step enqueues n_steps steps (asynchronous; the graph runs on a
 * stream of the batch ordered after and before the caller's stream).
 * kt_batch_tune chooses the flux kernel's block: per distinct grid shape its
 * cells in (x, y), 64 x 4, 32 x 8 or 16 x 16, then for the whole launch its
 * eta planes, 2 or 4.  It times the batched stage 1 (sources and flux
 * launches, all events together) on the live state, which it does not change:
 * every width of one shape with the other shapes held at their current choice
 * (shapes with the most cells first), then both plane counts; it keeps the
 * fastest, writes the choices per event (kc_out: eta planes, tile_out: the
 * block's width in x, 64, 32 or 16; each an array of n_events, nullable),
 * rebuilds the step and synchronises.  Results do not depend on the choice.
 * kt_batch_observables is kt_observables of one event.
 * --------------------------------------------------------------------- */
typedef struct kt_batch kt_batch;

size_t kt_batch_workspace_bytes(const kt_params *p, int32_t n_events, const kt_eos *eos);
kt_status kt_batch_init(const kt_params *p, int32_t n_events, const kt_eos *eos,
                        const kt_init_state *s0, void *d_ws, size_t ws_bytes, hipStream_t stream,
                        kt_batch **out);
kt_status kt_batch_step(kt_batch *b, int32_t n_steps);
kt_status kt_batch_tune(kt_batch *b, int32_t *kc_out, int32_t *tile_out);
/* Set the flux kernel's block per event without timing (for instance to reuse
 * an earlier kt_batch_tune result): kc[e] eta planes, 2 or 4 and the same for
 * every event; tile_x[e] in {64, 32, 16} cells in x (then 4, 8 or 16 cells in
 * y); arrays of n_events.  Rebuilds the step and synchronises; KT_E_ARG for
 * values outside these sets.  Results do not depend on the choice. */
kt_status kt_batch_set_flux_blocks(kt_batch *b, const int32_t *kc, const int32_t *tile_x);
kt_status kt_batch_observables(kt_batch *b, int32_t event, kt_obs *host_out, const kt_fields *dev_out);
void kt_batch_destroy(kt_batch *b);
const char *kt_batch_last_error(const kt_batch *b);

/* Release the context (not the workspace).  Null is allowed. */
void kt_destroy(kt_ctx *c);

/* Last error message of c, or of the calling thread when c is null. */
const char *kt_last_error(const kt_ctx *c);

const char *kt_status_string(kt_status s);

#ifdef __cplusplus
}
#endif

#endif /* KT_H */
