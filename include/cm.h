/*
 * cm.h -- C ABI of the MI355X (gfx950) nodal discontinuous-Galerkin LES hot
 * path: the right-hand side of the compressible Navier-Stokes equations with
 * total energy (and total water) as prognostic variables, and the explicit
 * low-storage Runge-Kutta step that calls it every stage.
 *
 * Method: Sridhar et al., "Large-eddy simulations with ClimateMachine",
 * GMD 2022 -- Sect. 2 (governing equations, Table 1, equation of state,
 * saturation adjustment), Sect. 3.1 (nodal GLL discretisation, mapping,
 * Rusanov flux eq. nonviscFlux, BR1 auxiliary gradient, semi-discrete
 * operator eq. matrixProblem), Sect. 3.2 (low-storage RK), Sect. 4 (SGS
 * closures eq. smago, eq. richardson), Sect. 6 (mass/energy integrals),
 * App. A (wall ghost states, prescribed wall fluxes, Rayleigh sponge).
 *
 * Conventions for every call:
 *  - State buffers (Y, Y_alt, dQ, dYdt) are caller-owned DEVICE memory on
 *    the grid's device, contiguous, layout [nvar][state_stride] with
 *    state_stride = 160*n_elem (cm_grid_info): element-major runs of 160
 *    slots, slot = 160*e + i + 5*(j + 5*k) for the node (i, j, k) of
 *    element e = ex + ne[0]*(ey + ne[1]*ez), i along x.  Slots 125..159 of a
 *    run are padding: never read as nodes, and written as zeros (125..127)
 *    or left untouched (128..159) in outputs.  The padding puts every
 *    element run on a 128-byte line in both precisions, so the kernels
 *    stream whole lines.  Element type double (CM_FP64) or float
 *    (CM_FP32_BULK), at least 16-byte aligned (256-byte for whole lines).
 *    The library never frees or retains them beyond a call.
 *  - What a state buffer holds: CM_FP64 models store full values;
 *    CM_FP32_BULK models store float(Y - Y_bg), each value's deviation from
 *    the model's background (cm_model_create), so that the FP32 rounding
 *    scales with the deviation and not with the hydrostatic background.
 *    cm_state_import / cm_state_export convert from and to full FP64
 *    values.  Tendencies (dQ, dYdt) are full values in both.
 *  - Grid and model objects own their device arrays (metrics, element
 *    traversal table, reference state, diffusive-flux scratch, the node
 *    temperatures moist viscous models carry between the passes and stages
 *    of a step, reduction scratch) and free them on destroy.
 *  - Compute calls are asynchronous on the hipStream_t passed as void*
 *    (NULL = the default stream).  Only create/copy calls and
 *    cm_diagnostics synchronise.
 *  - Every call returns a cm_status; on failure cm_last_error() returns a
 *    thread-local message.  No C++ exception crosses this boundary.  Calls
 *    on one model must not overlap on different streams.
 */
#ifndef CM_H
#define CM_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define CM_API __attribute__((visibility("default")))
#else
#define CM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CM_OK = 0,
    CM_ERR_ARG = 1,          /* invalid argument (null pointer, bad size, bad enum) */
    CM_ERR_HIP = 2,          /* a HIP runtime call failed */
    CM_ERR_ALLOC = 3,        /* device or host allocation failed */
    CM_ERR_UNSUPPORTED = 4,  /* valid but not implemented (e.g. N != 4) */
    CM_ERR_NONFINITE = 5,    /* cm_diagnostics found NaN/Inf in the state */
    CM_ERR_STATE = 6         /* object used in a wrong state (e.g. MLP closure without weights) */
} cm_status;

typedef enum { CM_FP64 = 0, CM_FP32_BULK = 1 } cm_precision;

typedef enum {
    CM_CLOSURE_NONE = 0,   /* inviscid */
    CM_CLOSURE_CONST = 1,  /* constant kinematic viscosity nu */
    CM_CLOSURE_SMAG = 2,   /* Smagorinsky-Lilly (eq. smago), optional Richardson factor */
    CM_CLOSURE_MLP = 3,    /* learned eddy viscosity / Prandtl number, Smagorinsky fallback */
    CM_CLOSURE_VREMAN = 4  /* Vreman (Sect. 4.2, eq. vreman-sgs), coefficient 2.5 Cs^2, mixing length
                              h_d / N per direction, optional Richardson factor */
} cm_closure;

/* Inviscid numerical flux n.F1* at element faces (Sect. 3.1).  Roe and HLLC
 * are for dry models (nvar = 5); a moist model with them fails to create
 * with CM_ERR_UNSUPPORTED. */
typedef enum {
    CM_FLUX_RUSANOV = 0,   /* centred + half the largest |u.n| + c times the jump */
    CM_FLUX_ROE = 1,       /* Roe: acoustic, entropy and shear waves of the sqrt(rho)-averaged state */
    CM_FLUX_HLLC = 2       /* HLLC: Davis wave-speed bounds, contact restored */
} cm_flux;

/* Mesh (Sect. 3.1): brick of ne[0] x ne[1] x ne[2] hexahedra over
 * [lo, hi]; periodic[d] != 0 wraps direction d, otherwise its two end faces
 * are free-slip walls.  topo = 1 warps the mesh terrain-following over the
 * Agnesi ridge z_sfc(x) = topo_h topo_a^2 / ((x - topo_xc)^2 + topo_a^2)
 * (eq. agnesi, Sect. 5.4) with linear decay to a flat lid at hi[2] (Sect. 5.3). */
typedef struct {
    int N;               /* polynomial order; only 4 is supported */
    int ne[3];
    double lo[3], hi[3]; /* metres */
    int periodic[3];
    int topo;            /* 0 flat, 1 Agnesi ridge along x */
    double topo_h, topo_a, topo_xc;
} cm_grid_desc;

typedef struct {
    int64_t n_elem;
    int64_t n_nodes;     /* 125 * n_elem (face nodes counted per element) */
    int N;
    int warped;
    double dmin_node;    /* minimum distance between adjacent GLL nodes [m] */
    int64_t state_stride; /* slots per variable in a state buffer: 160 * n_elem */
} cm_grid_info;

/* Physics of one model (Sects. 2, 4, App. A).  Units SI. */
typedef struct {
    int nvar;            /* 5: rho, rho u, rho v, rho w, rho e_tot; 6: + rho q_t */
    int precision;       /* cm_precision */
    int closure;         /* cm_closure */
    double nu;           /* CM_CLOSURE_CONST viscosity [m^2/s] */
    double Cs;           /* Smagorinsky coefficient */
    double Prt;          /* turbulent Prandtl number (1/3 in the paper) */
    int richardson;      /* multiply nu_t by the stability factor f_b(Ri) */
    double g;            /* gravity [m/s^2]; 0 disables gravity */
    double f_cor, u_g, v_g;            /* f-plane Coriolis and geostrophic wind */
    int sponge;                        /* Rayleigh sponge (eq. sponge) */
    double sp_zs, sp_ztop, sp_alpha, sp_gamma, sp_u[3];
    int sfc_flux;                      /* prescribed bottom fluxes (kinematic) */
    double theta_flux, qt_flux;        /* [K m/s], [m/s] */
    int subsidence;                    /* w_s = -w0 sin(pi z / z_top) acting on h_tot, q_t */
    double sub_w0, sub_ztop;
    int flux;                          /* inviscid numerical flux (Sect. 3.1): cm_flux */
    int ice;                           /* moist: the saturation adjustment splits the condensate between
                                          liquid and ice (Sect. 2.5, 2.7): liquid fraction 1 at and above
                                          273.15 K, 0 at and below 233 K, linear between; saturation over
                                          the mix weighted by it.  0: all liquid.  Ignored when dry. */
} cm_model_desc;

typedef struct {
    double mass, energy, water;  /* integrals of rho, rho e_tot, rho q_t (w_i w_j w_k |J|) */
    double ke;                   /* integral of |rho u|^2 / (2 rho) */
    double max_abs_w;            /* max |w| [m/s] */
    double max_cfl;              /* max (|u| + c) dt / dmin_node, 0 if dt <= 0 */
    double T_min, T_max;         /* temperature range [K] */
    int64_t n_nonfinite;         /* number of non-finite state entries */
} cm_diag;

typedef struct cm_grid cm_grid;
typedef struct cm_model cm_model;
typedef struct cm_mlp cm_mlp;

/* Build GLL nodes/weights and the differentiation matrix, node coordinates,
 * and (for warped meshes) per-node metric terms J a^d and 1/J from the
 * differentiated coordinates (Sect. 3.1 eq. mapping); uploads them to
 * hip_device.  *out owns its device arrays.
 * Errors: CM_ERR_ARG (null, ne < 1, hi <= lo), CM_ERR_UNSUPPORTED (N != 4,
 * or 16 x n_nodes >= 2^31: the kernels index nodes x words in 32 bits),
 * CM_ERR_HIP / CM_ERR_ALLOC. */
CM_API cm_status cm_grid_create(const cm_grid_desc* desc, int hip_device, cm_grid** out);
CM_API cm_status cm_grid_destroy(cm_grid* grid);
CM_API cm_status cm_grid_query(const cm_grid* grid, cm_grid_info* out);
/* Host copies: xyz_host [3][n_nodes]; wJ_host [n_nodes] = w_i w_j w_k |J|;
 * Ja_host [3 (d)][3 (component)][n_nodes] and J_host [n_nodes]. */
CM_API cm_status cm_grid_copy_coords(const cm_grid* grid, double* xyz_host);
CM_API cm_status cm_grid_copy_wJ(const cm_grid* grid, double* wJ_host);
CM_API cm_status cm_grid_copy_metrics(const cm_grid* grid, double* Ja_host, double* J_host);

/* Create a model on a grid.  Yref_host (host, [nvar][n_nodes], float64) is
 * the hydrostatic background; the library pushes it through its own
 * thermodynamics to obtain the reference pressure p_r and density rho_r
 * factored out of the momentum flux and the buoyancy (Sect. 2.4).  NULL
 * means p_r = rho_r = 0.  In CM_FP32_BULK the kernels evolve the stored
 * deviation about the background rounded to float (p_r and rho_r are
 * computed from that rounding), so that an imported state equal to Yref is
 * stored as exact zeros and is exactly at rest.
 * Errors: CM_ERR_ARG, CM_ERR_UNSUPPORTED (nvar not 5/6), CM_ERR_HIP/ALLOC. */
CM_API cm_status cm_model_create(const cm_grid* grid, const cm_model_desc* desc, const double* Yref_host,
                          cm_model** out);
/* Frees the model's device arrays.  Does not read the grid, so the grid may
 * be destroyed first (garbage collectors finalise in any order). */
CM_API cm_status cm_model_destroy(cm_model* model);

/* Learned closure weights for CM_CLOSURE_MLP (host, float32).  params: the
 * 9282 parameters of the 12-64-64-64-2 SiLU network, layer by layer, each
 * weight matrix row-major [out][in] followed by its bias.  norm: 48 floats:
 * input mean[12], std[12], then the standardised training range lo[12],
 * hi[12].  A node falls back to Smagorinsky when a standardised input leaves
 * the range widened by 10 % of its half-width on each side plus a margin of
 * 2^-20 (1 + |mean/std|) (the float rounding of the normalisation: an input
 * that was constant in training, such as the filter width on a uniform mesh,
 * passes at its training value), or when the network output is not finite.
 * Errors: CM_ERR_ARG (std <= 0 or hi < lo), CM_ERR_STATE (closure not MLP). */
CM_API cm_status cm_model_set_mlp(cm_model* model, const float* params_host, const float* norm_host);
/* number of node evaluations that fell back to Smagorinsky since the
 * previous call (each RHS evaluates every node once); resets the count.
 * Synchronises the stream. */
CM_API cm_status cm_model_mlp_fallbacks(cm_model* model, int64_t* count, void* hip_stream);

/* Closure inputs as the gradient pass computes them, for training the
 * learned closure: feat_dev (device, float64) [n_nodes][16] = grad u (9,
 * row i = component, column j = derivative direction), N^2, Delta,
 * (nu_SL / (0.1 Delta))^2, grad theta_v (3), theta_v.  Needs an FP64 model
 * with the Smagorinsky closure and the Richardson factor (CM_ERR_STATE
 * otherwise).  Asynchronous on the stream. */
CM_API cm_status cm_model_closure_inputs(cm_model* model, const void* Y, double* feat_dev, void* hip_stream);

/* dYdt = R(Y): the semi-discrete DG operator (eq. matrixProblem, strong
 * form) with F = F1 + F2, Rusanov F1*, centred F2*, BR1 gradients, closure,
 * sources.  Y and dYdt must not alias.  t is the model time (unused by the
 * present sources). */
CM_API cm_status cm_dg_rhs(cm_model* model, const void* Y, void* dYdt, double t, void* hip_stream);

/* One LSRK54 step (Carpenter-Kennedy 2N storage, 5 stages): for s = 1..5,
 * dQ = A_s dQ + dt R(Y_s, t + C_s dt); Y_{s+1} = Y_s + B_s dQ.  The stages
 * ping-pong Y -> Y_alt -> Y -> Y_alt -> Y -> Y_alt because neighbouring
 * elements still read the old state within a stage: on return the NEW state
 * is in Y_alt and Y holds an intermediate stage (swap the handles).  dQ need
 * not be initialised (A_1 = 0).  Y, Y_alt, dQ must be distinct. */
CM_API cm_status cm_lsrk_step(cm_model* model, void* Y, void* Y_alt, void* dQ, double t, double dt,
                       void* hip_stream);

/* One LSRK144 step (Sect. 3.2: the fourteen-stage fourth-order 2N-storage
 * scheme of Niegemann, Diehl & Busch, the paper's integrator for its
 * isotropic runs), the same fused stage update as cm_lsrk_step with its own
 * coefficients.  The stages ping-pong Y -> Y_alt -> Y ...; with fourteen
 * stages the NEW state ends in Y (Y_alt holds the thirteenth stage).  dQ need
 * not be initialised (A_1 = 0).  Y, Y_alt, dQ must be distinct.  Errors as
 * cm_lsrk_step. */
CM_API cm_status cm_lsrk144_step(cm_model* model, void* Y, void* Y_alt, void* dQ, double t, double dt,
                                 void* hip_stream);

/* 1-D IMEX ("HEVI", Sect. 3.2): horizontally explicit, vertically implicit
 * additive Runge-Kutta step for dry models (nvar = 5) on flat meshes with
 * walls at the bottom and top (CM_ERR_UNSUPPORTED otherwise).  The implicit
 * part L is the vertical acoustic operator linearised about the model's
 * background state (Yref_host of cm_model_create): on the deviation d = Y -
 * Y_ref, the vertical flux (rho w', p', h_r rho w'), with p' = (R_d/c_vd)
 * (rho e_tot)' + (R_d T_0 - (R_d/c_vd) g z) rho' and h_r = (rho e_r + p_r) /
 * rho_r, differentiated by the DG operator along xi3, the vertical part of
 * the Rusanov penalty at the background sound speed on all five variables,
 * mirrored ghosts at the walls, and the buoyancy -g rho'.  The explicit part
 * is cm_dg_rhs minus L.  Integrator: ARK2 of Giraldo, Kelly & Constantinescu
 * (2013), three stages, second order.  Each implicit stage solves (I - tau L)
 * d = B - Y_ref on every vertical node line (block-tridiagonal elimination
 * over the element layers, FP64).  When the background is horizontally
 * uniform (given per level), every line has the same matrix: the model then
 * keeps one factor of it, formed on the stream of the first solve with a
 * given tau and reused while tau stays the same (calls on one model must be
 * ordered, as for every model call); otherwise each line is eliminated on
 * its own.
 *
 * work: caller-owned device memory of cm_hevi_workspace_bytes bytes (six
 * state-sized buffers, the line solver's 60 doubles per element layer and
 * vertical node line, and two doubles per background entry), 256-byte
 * aligned; its contents need no initialisation and are scratch after the
 * call.  cm_hevi_step advances Y
 * in place by dt.  cm_hevi_operator writes L(Y - Y_ref) to LY (all five
 * variables).  cm_hevi_solve writes Y_ref + d with (I - tau L) d = B - Y_ref
 * to Y (B and Y may be the same buffer).  All asynchronous on the stream. */
CM_API cm_status cm_hevi_workspace_bytes(const cm_model* model, size_t* bytes);
CM_API cm_status cm_hevi_step(cm_model* model, void* Y, void* work, double t, double dt, void* hip_stream);
CM_API cm_status cm_hevi_operator(cm_model* model, const void* Y, void* LY, void* hip_stream);
CM_API cm_status cm_hevi_solve(cm_model* model, double tau, const void* B, void* Y, void* work, void* hip_stream);

/* Exponential modal filter (Sect. 5.4, eq. exponential_filter), in place on
 * the state Y (layout as cm_dg_rhs).  For each variable v with bit v set in
 * var_mask, each element's deviation from the model's background state
 * (Yref_host of cm_model_create; zero without one) is expanded in Legendre
 * modes along each direction, mode n is scaled by sigma(n) = exp(-alpha
 * ((n - Nc)/(N - Nc))^order) for n > Nc (by 1 for n <= Nc), and the
 * background is added back.  order is the filter order s (the paper uses
 * 64 on the velocity), alpha = -ln(machine epsilon) (36 in double
 * precision).  Mode 0 is never changed, so each element's integral of
 * every variable over its reference cube is kept; on flat meshes (constant
 * Jacobian) that is its physical integral.  Elements are filtered independently;
 * asynchronous on the stream.  Errors: CM_ERR_ARG (null, var_mask 0 or
 * beyond nvar bits, order < 1, alpha < 0 or not finite, Nc outside
 * 0 .. N-1). */
/* Stored state <-> full FP64 state.  cm_state_import writes the model's
 * storage of the full state Y_full into `state`; cm_state_export writes the
 * full values of `state` into Y_full.  Both buffers: caller-owned device
 * memory in the state layout above (Y_full double, `state` the model's
 * element type); padding slots of the output are written as zeros, those
 * of the input are not read.  For CM_FP64 the two are the same values
 * (the call copies; the buffers may coincide).  Asynchronous on the stream.
 * Errors: CM_ERR_ARG (null pointer). */
CM_API cm_status cm_state_import(cm_model* model, const double* Y_full, void* state, void* hip_stream);
CM_API cm_status cm_state_export(cm_model* model, const void* state, double* Y_full, void* hip_stream);

CM_API cm_status cm_exp_filter(cm_model* model, void* Y, int var_mask, int order, double alpha, int Nc,
                               void* hip_stream);

/* Conservation and health diagnostics (Sect. 6): compensated (Neumaier) FP64
 * integrals in a deterministic two-stage reduction, extrema, CFL and a
 * non-finite count.  Synchronises the stream.  Returns CM_ERR_NONFINITE
 * (with *out filled) when the state holds NaN/Inf. */
CM_API cm_status cm_diagnostics(cm_model* model, const void* Y, double dt, cm_diag* out_host, void* hip_stream);

/* cm_diagnostics for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid hipMalloc): the same reduction and
 * the same results, bit for bit, but its partial sums live in a static
 * per-device workspace of the library (2048 records of 16 doubles, 256 KiB,
 * held by every device the library runs on until the process ends) instead
 * of the model's, and the call makes no allocation.  The first pass strides
 * over the nodes with at most 2047 blocks, so the workspace bounds the
 * block count, not the grid: every grid cm_grid_create accepts fits, and a
 * node count outside 1 .. 2^27 fails with CM_ERR_ARG.  Nothing in the
 * workspace needs clearing (each call writes every record it reads).  All
 * calls on one device share the workspace: calls that overlap on one
 * device (different streams or threads) race and must be serialised by
 * the caller.  Synchronises the stream; CM_ERR_NONFINITE as cm_diagnostics. */
CM_API cm_status cm_diagnostics_noalloc(cm_model* model, const void* Y, double dt, cm_diag* out_host,
                                        void* hip_stream);

/* ---- learned closure training (12-64-64-64-2 SiLU MLP, BF16 MFMA, FP32
 * accumulate, FP32 master weights, Adam) ------------------------------- */
typedef struct {
    int n_in, n_hidden, n_layers_hidden, n_out;   /* must be 12, 64, 3, 2 */
    float lr, beta1, beta2, eps;                  /* Adam */
} cm_mlp_desc;

/* Initialise the network (uniform +-1/sqrt(fan_in) weights, zero biases) from
 * a 64-bit seed.  device buffers owned by the object. */
CM_API cm_status cm_mlp_create(const cm_mlp_desc* desc, uint64_t seed, int hip_device, cm_mlp** out);
CM_API cm_status cm_mlp_destroy(cm_mlp* mlp);
/* X_dev [batch][12] standardised inputs, T_dev [batch][2] targets (device,
 * float32).  One forward + backward + Adam update on the mean squared error;
 * *loss_host (if non-NULL) receives the batch loss (synchronises). */
CM_API cm_status cm_mlp_train_step(cm_mlp* mlp, const float* X_dev, const float* T_dev, int batch,
                            float* loss_host, void* hip_stream);
/* Gradient of the batch loss w.r.t. all 9282 parameters (host, float32). */
CM_API cm_status cm_mlp_grads(cm_mlp* mlp, const float* X_dev, const float* T_dev, int batch, float* grad_host,
                       void* hip_stream);
/* out_dev [batch][2] raw network outputs for standardised inputs. */
CM_API cm_status cm_mlp_infer(cm_mlp* mlp, const float* X_dev, float* out_dev, int batch, void* hip_stream);
CM_API cm_status cm_mlp_get_params(const cm_mlp* mlp, float* params_host);
CM_API cm_status cm_mlp_set_params(cm_mlp* mlp, const float* params_host);

/* Instrumentation: with profiling enabled the library brackets every kernel
 * launch of this model with a pair of hipEvents on the launch stream.
 * cm_model_profile(m, 1) starts (and clears) a record; read returns the
 * summed kernel durations [ms] and launch counts per kind: [0] gradient +
 * closure pass, [1] tendency pass (incl. the fused stage update).  The read
 * synchronises on the recorded events. */
CM_API cm_status cm_model_profile(cm_model* model, int enable);
CM_API cm_status cm_model_profile_read(cm_model* model, double* ms_host, int64_t* count_host);

CM_API const char* cm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CM_H */
