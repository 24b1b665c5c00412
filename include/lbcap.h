/*
 * lbcap — MI355X library for the D2Q9 free-energy multiple-relaxation-time
 * lattice Boltzmann scheme of Pooley, Kusumaatmaja & Yeomans, "Modelling
 * capillary filling dynamics using lattice Boltzmann simulations"
 * (arXiv:0911.0459): the van der Waals liquid-gas model (Sec. 2) and the
 * binary model with an order-parameter distribution (Sec. 3), in capillary
 * geometries (Sec. 2.2, Fig. 1b).
 *
 * Conventions shared by every entry point
 *  - Every call returns lb_status; LB_OK is 0, errors are negative.  A
 *    human-readable message for the last failing call of the calling thread is
 *    returned by lb_last_error().  No C++ exception crosses this interface.
 *  - Host arrays are owned by the caller.  Device state is owned by the
 *    library, unless a device allocation is handed in through d_state (then the
 *    caller owns that memory and must keep it alive until lb_free).
 *  - Work is enqueued on the HIP stream given at init (NULL: the library
 *    creates and owns a stream).  Calls that return host data synchronise that
 *    stream; lb_step and lb_batch_step only enqueue.
 *  - Lattice layout of every host field argument: ny*nx doubles, row-major,
 *    y major (index y*nx + x); x is the tube axis.
 *  - Units: lattice units, dx = dt = 1 (Sec. 2.1).
 *  - A context is not thread-safe; distinct contexts are independent.
 *
 * Geometry (Sec. 2.2, Fig. 1b).  The lattice is periodic in x.  A tube of
 * tube_h fluid rows [y0, y0+tube_h) occupies the columns [x_in, x_in+tube_len);
 * the rows above and below it in those columns are solid walls.  All other
 * nodes are reservoir, periodic in y.  tube_len = 0 means no walls at all.
 * Walls are no-slip: bounce-back plus "boundary nodes set to rest" after every
 * streaming step (Sec. 2.2).  Wetting is set by the normal gradient of rho
 * (vdW) or phi (binary) seen by the equilibrium at the wall (Sec. 2.2).
 */
#ifndef LBCAP_H
#define LBCAP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LB_OK = 0,
    LB_EINVAL = -1,     /* invalid argument: parameters, geometry, buffer size */
    LB_ENOMEM = -2,     /* device or host allocation failed */
    LB_EDEVICE = -3,    /* HIP runtime error (no device, launch failure) */
    LB_EUNSTABLE = -4,  /* non-finite value or non-positive density detected */
    LB_ESTATE = -5      /* call not valid in the context's current state */
} lb_status;

typedef enum { LB_VDW = 0, LB_BINARY = 1 } lb_model;

/* Model constants.
 *  vdW (Sec. 2, Eq. pt): p0 = rho T/(1 - b rho) - a rho^2, gradient coefficient kappa;
 *    the paper's values are kappa = 0.02, a = 9/49, b = 2/21, T = 0.56.
 *  binary (Sec. 3.1, Eq. chempot): mu = -A phi + B phi^3 - kappa lap(phi),
 *    p0 = rho/3 - A phi^2/2 + 3 B phi^4/4; the paper has A = B = kappa = 0.04.
 *  Gamma: coefficient 2M/dt of mu in g^eq (Appendix A); binary only.
 *  nu_l, nu_g: kinematic viscosities (Eq. nu; phi clamped to [-1, 1]); the
 *    relaxation rate is omega = 2/(6 nu + 1) (Appendix A).  vdW uses nu_l.
 *  wall_grad: normal derivative of rho/phi at the wall, normal into the fluid;
 *    negative is hydrophilic.  Used when theta_deg is NaN.
 *  theta_deg: equilibrium contact angle; when not NaN, wall_grad is computed
 *    with lb_wall_gradient_for_angle.
 *  force_x: uniform body force along x (Guo, Zheng & Shi 2002 forcing in
 *    moment space); acts on fluid nodes that are not boundary nodes.
 *  lambda_mode: 0 gives the Galilean-correction term of Eq. (equilibrium)
 *    (vdW) the Chapman-Enskog coefficients of the Appendix A rates: its
 *    traceless part (1/omega - 1/2)(1/3 - dp0/drho), relaxed with the stresses
 *    at omega, and its isotropic part (1/2)(1/3 - dp0/drho), relaxed with the
 *    energy moment at rate 1 (one lambda when omega = 1, as printed); this is
 *    what keeps a translating interface moving with the fluid.  1 sets
 *    lambda = 0.  The binary model always uses lambda = 0.
 *  q_mid: level of rho/phi that marks the interface for the filled length;
 *    NaN selects 0 (binary) or the mean of the Maxwell coexistence densities
 *    of p0 (vdW). */
typedef struct {
    lb_model model;
    double kappa, a, b, T;
    double A, B, Gamma;
    double nu_l, nu_g;
    double wall_grad;
    double theta_deg;
    double force_x;
    int lambda_mode;
    double q_mid;
} lb_params;

typedef struct {
    int nx, ny;
    int x_in, tube_len;
    int tube_h, y0;
} lb_geometry;

typedef struct lb_ctx lb_ctx;

/* Message of the last failing call on this thread ("" if none). */
const char* lb_last_error(void);

/* Device bytes needed by lb_init for these parameters and this geometry
 * (two FP32 population buffers, descriptors, tile table, l(t) history).
 * Returns 0 for invalid arguments. */
size_t lb_state_bytes(const lb_params* p, const lb_geometry* g);

/* Create a single-lattice context at t = 0 (Sec. 2.2 / 3.2 setups).
 *  init_q: host, ny*nx doubles: the initial rho (vdW) or phi (binary, rho = 1),
 *    noise included; values at solid nodes are ignored.  The populations start
 *    at equilibrium with u = 0 (f = f^eq, g = g^eq, Appendix A).
 *  d_state/bytes: optional device allocation of at least lb_state_bytes()
 *    bytes, 256-byte aligned (e.g. from PyTorch); NULL lets the library allocate.
 *  hip_stream: hipStream_t to enqueue on; NULL creates a library-owned stream.
 * Validation: 0 < omega < 2 for every viscosity, 0 < b rho < 1 for vdW,
 * |phi| < 3.5 for the binary model (phi is stored as a 32-bit fixed-point
 * number with 29 fraction bits, range 4, so that the small updates in the
 * tails of an interface are kept), finite values, H >= 3, 1 <= y0,
 * y0 + H <= ny - 1, x_in + tube_len <= nx, Gamma >= 0.
 * Errors: LB_EINVAL, LB_ENOMEM, LB_EDEVICE. */
lb_status lb_init(lb_ctx** out, const lb_params* p, const lb_geometry* g, const double* init_q,
                  void* d_state, size_t bytes, void* hip_stream);

/* Advance nsteps time steps of Eq. (latbolt) (and Eq. (latbolt2) for the
 * binary model): moments, stencils of Eq. (best), equilibria, MRT collision
 * with the rates of Appendix A, streaming with bounce-back, rest of boundary
 * nodes.  Asynchronous; errors of the launches are reported here, a numerical
 * blow-up by lb_check or the next call that reads data back. */
lb_status lb_step(lb_ctx* c, long nsteps);

/* Number of steps taken since lb_init / lb_load. */
long lb_time(const lb_ctx* c);

/* Scan every fluid node for a non-finite population or rho <= 0; synchronises.
 * Returns LB_EUNSTABLE (latched for the context) if one is found. */
lb_status lb_check(lb_ctx* c);

/* Macroscopic fields at the current time into caller-owned host arrays of
 * ny*nx doubles (any may be NULL): rho, u = (j + F/2)/rho, phi (binary; 0 for
 * vdW).  Solid nodes get 0.  Synchronises. */
lb_status lb_moments(lb_ctx* c, double* rho, double* ux, double* uy, double* phi);

/* Same fields as FP32 into caller-owned device arrays of ny*nx floats (any may
 * be NULL).  Enqueued on the context stream, no synchronisation. */
lb_status lb_moments_device(lb_ctx* c, float* rho, float* ux, float* uy, float* phi);

/* Filled length l (Fig. 1b) and l_eff = l + H/2 (Sec. 3.2) at the current time:
 * q on the tube centreline (mean of the two middle rows for even H) is scanned
 * from x_in; l is the linearly interpolated first position where q drops below
 * q_mid (0 if the first tube node is already below, tube_len if never).
 * Synchronises.  LB_EINVAL if the geometry has no tube. */
lb_status lb_interface_length(lb_ctx* c, double* l, double* l_eff);

/* Contact angle of the meniscus in the tube (Sec. 3.2, Fig. 5): in every tube
 * row except edge_rows rows next to each wall, the interface is the first
 * position from the inlet where q (phi, or rho for vdW) falls below q_mid,
 * linearly interpolated (rows with no liquid at the inlet are skipped).  A
 * circle centred on the channel centreline is fitted to these points by linear
 * least squares; with the walls half a node outside the boundary rows the
 * channel is H wide and cos(theta) = (H/2)/R, positive when the centre lies on
 * the gas side.  theta_deg is measured through the liquid (liquid on the inlet
 * side), radius is R (INFINITY for a flat interface), apex_x the interface
 * position on the centreline; each output pointer may be NULL.
 * lb_meniscus_angle_field works on a caller-owned host field q (ny x nx,
 * row-major) and needs no device; lb_meniscus_angle reads capillary cap of a
 * context (synchronises).  LB_EINVAL: no tube, edge_rows leaves fewer than 3
 * rows; LB_ESTATE: fewer than 3 rows hold an interface. */
lb_status lb_meniscus_angle_field(const double* q, const lb_geometry* g, double q_mid, int edge_rows,
                                  double* theta_deg, double* radius, double* apex_x);
lb_status lb_meniscus_angle(lb_ctx* c, int cap, int edge_rows, double* theta_deg, double* radius,
                            double* apex_x);

/* Flow along the tube (Sec. 2.2, Fig. 3).  From host fields (ny x nx,
 * row-major) q (rho for vdW, phi for binary: locates the meniscus), rho and u_x:
 *  u_centre (caller-owned, tube_len doubles, may be NULL): u_x on the tube
 *    centreline (mean of the two middle rows for even H) at x_in .. x_in+tube_len-1;
 *  out->l: the filled length, as lb_interface_length, from q and q_mid;
 *  out->rho_liquid, u_liquid: mean density and mass-weighted mean x velocity
 *    sum(rho u_x)/sum(rho) of the channel rows from x_in + margin to the
 *    meniscus minus margin (the liquid column; liquid_cols columns);
 *  out->rho_gas, u_gas: the same from the meniscus plus margin to the tube's
 *    end minus margin (the gas ahead; gas_cols columns);
 *  out->condensation_liquid_side = rho_liquid (v_meniscus - u_liquid) and
 *  out->condensation_gas_side = rho_gas (v_meniscus - u_gas): the mass that
 *    crosses the moving meniscus per unit time and width, seen from either
 *    side (positive: the gas condenses); equal for a steady interface.
 *    v_meniscus is the meniscus speed dl/dt, e.g. from two filled lengths.
 * lb_tube_flow reads capillary cap of a context with its own q_mid
 * (synchronises).  LB_EINVAL: no tube, margin < 0, non-finite q_mid or
 * v_meniscus. */
typedef struct {
    double l;
    double rho_liquid, u_liquid;
    double rho_gas, u_gas;
    double condensation_liquid_side, condensation_gas_side;
    int liquid_cols, gas_cols;
} lb_tube_flow_stats;
lb_status lb_tube_flow_field(const double* q, const double* rho, const double* ux, const lb_geometry* g,
                             double q_mid, int margin, double v_meniscus, double* u_centre, lb_tube_flow_stats* out);
lb_status lb_tube_flow(lb_ctx* c, int cap, int margin, double v_meniscus, double* u_centre,
                       lb_tube_flow_stats* out);

/* Filled length l(t) by the capillary balance of Eq. 1 - 3 with the viscous
 * drag of the liquid column (dynamic viscosity eta_l) and of the gas column of
 * length L - l ahead of it (eta_g): the solution of
 *   (eta_l - eta_g) (l^2 - l0^2) / 2 + eta_g L (l - l0) = gamma H cos(theta) t / 6
 * continuous with l(0) = l0 (Sec. 2.2, Fig. "10", dashed and dotted lines);
 * eta_g = 0 is Washburn's law, Eq. 3.  Host arithmetic, no device.
 * LB_EINVAL for t < 0, l0 outside [0, L], H <= 0, eta_l <= 0, eta_g < 0. */
lb_status lb_washburn_length(double t, double l0, double H, double L, double gamma, double cos_theta,
                             double eta_l, double eta_g, double* l);

/* Wall gradient that gives the equilibrium contact angle theta_deg by Young's
 * law (Eq. Young) with the surface tensions of the Cahn construction for a
 * surface energy linear in the wall value of rho/phi (Sec. 2.2, Fig. 2).
 * Binary model: closed form in the bulk values +-sqrt(A/B).  vdW model:
 * numerical quadrature of the van der Waals free energy at coexistence.
 * theta in (0, 180); LB_EINVAL outside the partial-wetting range. */
lb_status lb_wall_gradient_for_angle(const lb_params* p, double theta_deg, double* grad);

/* Change the wall gradient of capillary cap (normal derivative of rho/phi at
 * the wall, normal into the fluid) for the steps that follow: the equilibrium
 * gradient scanned slowly in time gives the contact angle as a function of the
 * gradient (Sec. 2.2, Fig. 2).  grad must be finite (LB_EINVAL otherwise).
 * The library stores post-collision populations: at time T the collision of
 * time T has been evaluated, so the new gradient enters from the collision of
 * time T+1 on (one step after a scheme that stores the streamed state).
 * Synchronises the context stream; captured graphs stay valid (the kernels
 * read the gradient from the device descriptor).  The parameter hash of checkpoints
 * includes the gradient: an image saved at another gradient is refused. */
lb_status lb_set_wall_gradient(lb_ctx* c, int cap, double grad);

/* Coexisting densities of the van der Waals p0 (equal pressure and chemical
 * potential, the Maxwell construction) for the constants in p. */
lb_status lb_vdw_coexistence(const lb_params* p, double* rho_l, double* rho_g);

/* Checkpoint: bytes needed, save into / restore from a caller-owned host
 * buffer.  The image holds the populations, the step count and a hash of the
 * parameters and geometry; lb_load refuses an image of another setup
 * (LB_EINVAL).  Resuming is bitwise identical to not stopping.  The image
 * records the storage of schedule 6 or of the others; an image of the other
 * storage is converted on load (then equal to rounding). */
size_t    lb_checkpoint_bytes(const lb_ctx* c);
lb_status lb_save(lb_ctx* c, void* host_buf, size_t bytes);
lb_status lb_load(lb_ctx* c, const void* host_buf, size_t bytes);

/* Release the context (its stream and allocations, not a caller's d_state). */
void lb_free(lb_ctx* c);

/* ---- batches of capillaries (one launch per step advances all of them) ----
 * n capillaries, each with its own parameters and geometry (all of the same
 * model), advance together: every time step is one kernel launch over the
 * tiles of all lattices, and runs of steps are replayed from HIP graphs.
 * Capillary k is addressed by its index 0..n-1. */
lb_status lb_batch_init(lb_ctx** out, int n, const lb_params* p, const lb_geometry* g,
                        const double* const* init_q, void* hip_stream);

/* Advance every active capillary by nsteps.  If sample_every > 0 the filled
 * length l_eff of each active capillary is appended to its device history
 * whenever the step count becomes a multiple of sample_every (capacity
 * LB_HISTORY_CAP samples; later samples are dropped and reported by
 * lb_batch_l_history).  Asynchronous. */
lb_status lb_batch_step(lb_ctx* c, long nsteps, int sample_every);

#define LB_HISTORY_CAP 4096

/* Copy capillary cap's l_eff history into host array l (at most max_samples)
 * and its length into *n_samples (may exceed max_samples).  Also fills the
 * step count of each sample into steps if not NULL.  Synchronises. */
lb_status lb_batch_l_history(lb_ctx* c, int cap, double* l, long* steps, int max_samples,
                             int* n_samples);

/* Stop advancing capillary cap (accepted by the surrogate gate or failed);
 * its state is frozen.  lb_batch_revive undoes it. */
lb_status lb_batch_retire(lb_ctx* c, int cap);
lb_status lb_batch_revive(lb_ctx* c, int cap);

/* Host fields of one capillary of a batch, as lb_moments.  Synchronises. */
lb_status lb_batch_moments(lb_ctx* c, int cap, double* rho, double* ux, double* uy, double* phi);

/* Per-capillary health flags after a scan (0 ok, 1 unstable); synchronises.
 * flags: host array of n ints. */
lb_status lb_batch_health(lb_ctx* c, int* flags);

/* Number of capillaries and of fluid nodes in the context. */
int       lb_batch_size(const lb_ctx* c);
long long lb_fluid_nodes(const lb_ctx* c);

/* Launch configuration of the step kernel.
 *  schedule: 3 row-sweep strips: one wavefront per strip of 62
 *    output columns marching along y through chunks of chunk_rows rows (0: the
 *    whole height), strips grouped so that each of the 8 XCDs works on a
 *    contiguous run of them; every population row is read once per step.
 *    4 (the van der Waals model's default) the same row sweep with a workgroup per strip of 192 output columns
 *    aligned to the row pitch (three wavefronts of 64 output columns and one
 *    that supplies the two neighbour columns), so that no stored cache line is
 *    shared between workgroups.  The same arithmetic as 3, compiled apart:
 *    the results agree to the last bits (vdW bitwise, binary within 3e-7).
 *    5 the strips of 4, each launch advancing two time steps: the sweep
 *    reads the populations (and phi) once with a halo of three nodes (binary
 *    model: four), keeps the intermediate step in LDS and writes the second
 *    step, so that the populations cross HBM once per two steps; an odd step
 *    count ends with one launch of schedule 4, and with the binary model every
 *    stepping call does (the read-outs take phi of the step the last launch
 *    read, which a two-step launch leaves one step behind).  The same
 *    arithmetic per step as schedule 4 (the intermediate step rounded to
 *    FP32, phi to its fixed point, as a single step stores them): van der
 *    Waals results are bitwise those of schedule 4, binary ones agree to
 *    rounding.
 *    6 (binary model only; its default) the strips of 4 over a stored state of seven FP32
 *    planes instead of nine populations: with the rates of Appendix A the
 *    post-collision populations of a node follow from rho - rho_ref, j* / 3, the
 *    common parts of the axis and of the diagonal populations, pxx* and pxy*,
 *    so a step moves 32 instead of 40 bytes per node (phi included).  The
 *    sweep rebuilds the populations of each row once, into LDS, and pulls
 *    from there.  Setting this schedule converts the stored state in place
 *    (both buffers); leaving it converts back (a context of the binary model
 *    starts in it).  Results agree with schedule 4
 *    to rounding (the populations are rebuilt in FP32 from the stored FP32
 *    state instead of being rounded once from the collision's arithmetic).
 *    0..2 tiles of 64 x tile_rows nodes with the order field recomputed on a
 *    halo: 0 one workgroup per tile in table order, 1 tiles grouped per XCD,
 *    2 persistent workgroups (persist_blocks_per_cu x 256 CUs) striding the table.
 *  tile_rows: rows per tile for schedules 0..2 (1, 2, 4 or 8).
 *  chunk_rows: target rows per strip chunk for schedules 3..6 (0, or 4..4096;
 *    default 8 for the van der Waals model, 20 for the binary one): each strip column is cut into chunks of about that height that
 *    start an even number of rows apart, so that the results do not depend on it.
 *    From 12 rows on, the last rows of the last columns of each XCD's run go to
 *    short chunks (a quarter of the height, at least 4 rows) that end the step.
 *  graph_steps: time steps captured per HIP graph (even, >= 2; 0 = no graphs).
 *  fp64_arith: 0 (default) evaluates the collision in FP32; 1 evaluates its
 *    non-shear part in FP64 (schedules 3..6; schedules 0..2 then compute the
 *    whole step in FP64).  In FP32 the j/3 of the populations is formed with a
 *    correction of its rounding (the rounded 1/3 would amplify the streamed
 *    momentum every step); with it both settings hold the 10^4-step oracle
 *    gates equally.  The stored state is FP32 either way (same memory
 *    traffic). */
typedef struct {
    int tile_rows;
    int schedule;
    int persist_blocks_per_cu;
    int graph_steps;
    int fp64_arith;
    int chunk_rows;
} lb_launch_config;

lb_status lb_get_launch_config(const lb_ctx* c, lb_launch_config* cfg);
lb_status lb_set_launch_config(lb_ctx* c, const lb_launch_config* cfg);

/* Autotuner: times the candidate launch configurations on this context's own
 * lattices (each for `trial_steps` steps, state restored afterwards), keeps
 * the fastest and returns it with its time per step in microseconds.  The
 * arithmetic (fp64_arith) is not tuned: candidates keep the context's value.
 * The shape found is also remembered for this process, per model and size
 * class (floor(log2) of the number of fluid nodes). */
lb_status lb_autotune(lb_ctx* c, int trial_steps, lb_launch_config* best, double* us_per_step);

/* Apply the launch shape last tuned in this process for the context's model
 * and size class, if any (*found = 1; else 0 and nothing changes).  Only the
 * shape fields are taken (schedule, tile_rows, chunk_rows,
 * persist_blocks_per_cu, graph_steps); fp64_arith stays the context's own.
 * A context never takes a tuned shape by itself: it starts from the default
 * configuration, so its results do not depend on what was tuned before it. */
lb_status lb_use_tuned_launch_config(lb_ctx* c, int* found);

/* Average duration (microseconds) of the step kernel over the launches
 * enqueued by the last lb_step / lb_batch_step call, measured with HIP events
 * on the context stream (0 if not available).  Synchronises. */
lb_status lb_last_step_kernel_us(lb_ctx* c, double* us);

/* Device-to-device copy of `bytes` (a multiple of 16, 16-byte aligned
 * pointers) by a plain kernel with one 16-byte load and store per thread,
 * enqueued on hip_stream.  Measurement infrastructure, not part of the
 * method: it is the achievable-bandwidth reference for the step kernel's
 * roofline and the kernel of known traffic that calibrates the HBM byte
 * counters (its callers are the benchmark and the profiling runs). */
lb_status lb_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

/* ---- learned l(t) surrogate: MLP 19 -> 256 -> 256 -> 256 -> 64, GELU ----
 * Hand-written HIP kernels for the forward pass, the backward pass and Adam
 * (Kingma & Ba 2015), FP32, parameters resident on the device.
 * Inputs and outputs are caller-owned host FP32 arrays, row-major, one row per
 * sample (n x 19 in, n x 64 out). */
typedef struct mlp_net mlp_net;

lb_status mlp_init(mlp_net** out, int seed, void* hip_stream);
void      mlp_free(mlp_net* net);
/* Number of FP32 parameters (153152 for this architecture). */
long      mlp_param_count(const mlp_net* net);
/* Copy parameters (W1,b1,W2,b2,W3,b3,W4,b4; W is out x in row-major) to/from host. */
lb_status mlp_get_params(mlp_net* net, float* host, long count);
lb_status mlp_set_params(mlp_net* net, const float* host, long count);
/* Forward pass for n rows. */
lb_status mlp_predict(mlp_net* net, const float* X, int n, float* Y);
/* Allocation-free forward pass, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same outputs as mlp_predict, from caller-owned
 * DEVICE arrays X (n x 19) and Y (n x 64, written), enqueued on the network's
 * stream without synchronising.  No allocation: the hidden activations live
 * in a static device array of 3 x MLP_NOALLOC_MAX_ROWS x 256 floats (3 MiB)
 * that each GPU holds until the process ends; n above MLP_NOALLOC_MAX_ROWS is
 * rejected with LB_EINVAL.  Every call on one GPU uses the same array, so calls
 * that overlap in time on one GPU (other streams, other threads, other
 * networks) race and must be serialised by the caller. */
#define MLP_NOALLOC_MAX_ROWS 1024
lb_status mlp_predict_device_noalloc(mlp_net* net, const float* X, int n, float* Y);
/* Mean-squared-error loss and its parameter gradient for n rows (no update);
 * grads has mlp_param_count floats in the mlp_get_params layout. */
lb_status mlp_loss_grad(mlp_net* net, const float* X, const float* Y, int n, float* loss,
                        float* grads);
/* Train with Adam (beta1 0.9, beta2 0.999, eps 1e-8) on minibatches of
 * `batch` rows drawn in a seeded shuffled order, for `epochs` passes.
 * Writes the mean loss of the last epoch into *last_loss if not NULL. */
lb_status mlp_train(mlp_net* net, const float* X, const float* Y, int n, int epochs, int batch,
                    float lr, int seed, float* last_loss);

#ifdef __cplusplus
}
#endif
#endif
