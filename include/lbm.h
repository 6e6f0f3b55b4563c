/*
 * lbm.h - C ABI of the MI355X (gfx950) reactive colour-gradient lattice Boltzmann step.
 *
 * Method: J.M.P. Beunen and J. Harting, "Gas-generating reactive flows in bicontinuous catalyst
 * support structures". One call of lbm_step advances the two-colour D3Q19 colour-gradient model
 * (Sec. II.A) by one time step per iteration: pull streaming with halfway bounce-back (eq.
 * bounce_back) and periodic faces, the generalized central-moments collision (Appendix A, eqs.
 * collision_operator .. back_transformation_vector), exact-difference forcing (eq.
 * operator_perturbation) with the continuum-surface-force surface tension (eqs.
 * continuum_surface_force, interface_curvature, color_gradient_normal, finite_difference_scheme),
 * Latva-Kokko recolouring (eq. operator_recoloring), Akai wetting (eqs.
 * color_lattice_weighted_average, realigned_normal_vectors, normal_vector_solid) and the
 * first-order wall reaction that turns reactant (red) into product (gas) colour (eqs.
 * nearest_solid_neighbors, reactive_boundary_condition_reactant/product). An optional D3Q7
 * advection-diffusion species (not in the paper) is consumed by the same wall reaction.
 *
 * Conventions shared by every entry point:
 *   - Node (x, y, z) has linear index n = x + nx*(y + ny*z); arrays of per-node vectors are
 *     stored component-major: component a of node n at [a*N + n], N = nx*ny*nz.
 *   - "Host" pointers are ordinary CPU memory, read during the call and not retained.
 *     "Device" pointers are HIP device memory owned by the caller; the library borrows them
 *     for the lifetime stated and never frees them.
 *   - All work is ordered on the HIP stream given to lbm_init. Entry points that return host
 *     data (reductions) synchronize that stream before returning.
 *   - Real-valued device outputs use the context's real type: double when precision is
 *     LBM_FP64, float otherwise.
 *   - No call aborts or throws: every error is a negative lbm_status, with a message from
 *     lbm_last_error(ctx). On an error the context's state is left as it was before the call
 *     unless stated otherwise.
 *   - Contact angles are in radians, measured through the red (reactant) colour.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_ERR_ARG = -1,         /* invalid argument (value, size, null pointer, too-small buffer) */
  LBM_ERR_ALLOC = -2,       /* host allocation failed */
  LBM_ERR_HIP = -3,         /* a HIP runtime call failed (message holds the HIP error string) */
  LBM_ERR_NONFINITE = -4,   /* a step produced a non-finite value; state is kept for inspection */
  LBM_ERR_STATE = -5,       /* call not valid in the context's current state */
  LBM_ERR_UNSUPPORTED = -6  /* option combination not supported */
} lbm_status;

/* Storage precision of the populations. Arithmetic is FP64 for LBM_FP64 and FP32 otherwise;
 * the five global reductions are always accumulated in FP64. The *_DEV modes store each
 * population as its deviation from the lattice weight, scaled by 2^fp16_scale_log2 (FP16) or
 * unscaled (BF16). */
typedef enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16_DEV = 2, LBM_BF16_DEV = 3 } lbm_precision;

typedef struct lbm_ctx lbm_ctx; /* opaque */

/* Problem statement (Sec. II and Sec. IV.B of the paper). */
typedef struct {
  int32_t nx, ny, nz;      /* lattice size, each >= 1, nx*ny*nz < 2^31 */
  int32_t precision;       /* lbm_precision */
  int32_t species;         /* 0: paper's model, reaction with C = 1; 1: D3Q7 species on */
  int32_t x_open;          /* species only: inlet at x = 0 (C = c_inlet), outflow at x = nx-1;
                            * needs nx >= 2 */
  double tau;              /* relaxation time of the shear central moments, > 0.5 (eq. kinematic_viscosity) */
  double tau_species;      /* species BGK relaxation time, > 0.5 (D = (tau_species - 1/2)/4) */
  double sigma;            /* surface tension sigma >= 0 (eq. continuum_surface_force) */
  double beta;             /* recolouring parameter beta >= 0 (eq. operator_recoloring) */
  double xi;               /* reaction rate xi >= 0 (eq. reactive_boundary_condition_reactant) */
  double accel[2][3];      /* body acceleration a^k of red (k = 0) and product (k = 1) */
  double c_inlet;          /* species inlet concentration (x_open) */
  double grad_eps;         /* colour gradients with |grad rho^N| <= grad_eps give n = 0; > 0 */
  int32_t fp16_scale_log2; /* deviation scale exponent for LBM_FP16_DEV, 0..20 */
  int32_t fluid_nodes;     /* number of fluid nodes of the mask, which sizes the state and adjoint
                            * planes and the per-fluid-node arrays (half the memory of an every-node
                            * layout at porosity 0.5); 0 sizes them for every node. Every size query
                            * and lbm_init must see the same value; lbm_init rejects a mask whose
                            * fluid count differs. 0..nx*ny*nz */
} lbm_params;

/* Level-t sums of one step (eqs. reactant_mass, product_mass, production_rate), in FP64:
 * m^r = sum rho^r, m^p = sum rho^p, conversion = sum of converted red mass, species_total =
 * sum C, nonfinite = number of fluid nodes with a non-finite result. */
typedef struct {
  double mass_r, mass_p, conversion, species_total, nonfinite;
} lbm_reductions;

/* Library version string (static storage). */
const char* lbm_version(void);

/* Bytes of device workspace that lbm_init needs for these parameters. */
lbm_status lbm_workspace_bytes(const lbm_params* params, size_t* bytes);

/* Bytes of one opaque state snapshot (lbm_get_state / lbm_set_state / lbm_adjoint_step). */
lbm_status lbm_state_bytes(const lbm_params* params, size_t* bytes);

/* Creates a context and writes the initial state S_0 = f^eq(rho^k_0, 0) per colour (and
 * g = w C_0 for the species). Host inputs, N values each:
 *   solid     uint8, 1 = solid node, 0 = fluid (required)
 *   theta     double, contact angle in [0, pi] per node (read at wetting nodes); NULL = use
 *             theta_uniform everywhere
 *   reactive  uint8 r(x) (1 = reaction active); NULL = every fluid node with a solid face
 *             neighbour (NN > 0)
 *   rho_r0, rho_p0  double, initial colour densities (read at fluid nodes, rho_r0 + rho_p0 > 0)
 *   c0        double initial species concentration; NULL = 1 (ignored without species)
 * d_workspace: device memory of at least lbm_workspace_bytes, 256-byte aligned, owned by the
 * caller and used by the context until lbm_free. stream: hipStream_t or NULL (default stream).
 * Errors: LBM_ERR_ARG for invalid parameters or inputs (tau <= 0.5, negative sigma/beta/xi,
 * theta outside [0, pi], non-finite values, non-positive mixture density at a fluid node,
 * misaligned or too small workspace, params->fluid_nodes > 0 differing from the mask's fluid
 * count); LBM_ERR_HIP. *out is set only on success. */
lbm_status lbm_init(const lbm_params* params, const uint8_t* solid, const double* theta, double theta_uniform,
                    const uint8_t* reactive, const double* rho_r0, const double* rho_p0, const double* c0,
                    void* d_workspace, size_t workspace_bytes, void* stream, lbm_ctx** out);

/* Advances nsteps >= 0 time steps on the context's stream. per_step: host array of nsteps
 * lbm_reductions (level t of each step) or NULL. Synchronizes the stream before returning.
 * Returns LBM_ERR_NONFINITE if any step counted a non-finite node (the state after the
 * last step is kept). */
lbm_status lbm_step(lbm_ctx* ctx, int32_t nsteps, lbm_reductions* per_step);

/* The same nsteps >= 0 time steps, only enqueued on the context's stream: returns without
 * waiting, computes no host-visible reductions and does not report non-finite values (the step
 * kernels are the ones lbm_step launches, so the state is bitwise the same). For drivers that
 * keep the stream busy, such as the recomputation of a checkpoint segment. Kernel timing
 * (lbm_set_profiling) does not cover these steps. Errors: LBM_ERR_ARG, LBM_ERR_HIP. */
lbm_status lbm_step_async(lbm_ctx* ctx, int32_t nsteps);

/* Level-t fields of the current state without changing it (steps up to the forcing of the
 * next update): rho^r, rho^p, rho^N (N each), the physical velocity u + F/(2 rho^m)
 * (3N, component-major) and the species concentration C (N; 1 without species). Device
 * pointers of the context's real type; any may be NULL. Solid nodes receive 0. */
lbm_status lbm_moments(lbm_ctx* ctx, void* d_rho_r, void* d_rho_p, void* d_rho_n, void* d_u, void* d_c);

/* The post-collision populations S_t per colour, expanded from the internal representation:
 * d_fr, d_fp (19N each, population-major [i*N + n], lattice order of the paper's matrix M with
 * the rest vector last) and d_g (7N, order +x,-x,+y,-y,+z,-z,rest; may be NULL). Device
 * pointers of the context's real type. Solid nodes receive 0. */
lbm_status lbm_populations(lbm_ctx* ctx, void* d_fr, void* d_fp, void* d_g);

/* Static geometry computed at init, for inspection: d_info (uint32 N) holds, at fluid nodes,
 * bit i (i < 18) = node x - c_i is solid, bit 18 = fluid, bit 19 = wetting node (some
 * neighbour solid), bits 20..22 = r(x) * NN(x); at solid nodes bit i (i < 18) = node x + c_i
 * is fluid and bit 23 = colour is extrapolated into this node. d_wet (4N, real type, node-major
 * [4*n + k]): at fluid nodes the unit solid normal n_s (k = 0..2, zero where undefined) and
 * cos(theta) (k = 3); zero at solid nodes. Either may be NULL. */
lbm_status lbm_geometry(lbm_ctx* ctx, void* d_info, void* d_wet);

/* Byte offsets inside a state snapshot of its three parts, and the plane stride P (elements;
 * P >= F, F = params->fluid_nodes, or N when that is 0, padded so that planes are an odd multiple
 * of 256 bytes apart): the 19 colour-blind
 * population planes f^m (storage type, population-major [i*P + f]), the colour scalars as one
 * 4-vector per node (e, v_x, v_y, v_z; real type, [4*f + k]) and the 7 species planes (storage
 * type, [i*P + f]; absent without species). The per-colour populations are
 * f^r_i = a f^m_i + (w_i/|c_i|) c_i.v and f^p_i = b f^m_i - (w_i/|c_i|) c_i.v with a + b = 1;
 * e holds the smaller of a and b at full precision: e = -b when the sign bit of e is set
 * (e = -0: pure reactant colour), else e = a. The state holds fluid nodes only: f is the fluid
 * id, the rank of the node among the fluid nodes in node order (0 .. nfluid-1); entries
 * f >= nfluid are unused. In the *_DEV storages a population f is stored as (f - w_i) * 2^k
 * (k = fp16_scale_log2 for FP16, 0 for BF16); their species part is each node's species total C
 * (real type, one per fluid id, at g_off plus the 7 planes rounded up to 256 bytes) and the 7
 * populations as (g_q - w_q C) * 2^k. Any output pointer may be NULL. */
lbm_status lbm_state_layout(const lbm_params* params, size_t* f_off, size_t* a_off, size_t* g_off,
                            size_t* plane_stride);

/* Copies the current state (lbm_state_bytes) to / from caller device memory, stream-ordered.
 * Together with lbm_steps_done this is a bitwise-exact checkpoint. */
lbm_status lbm_get_state(lbm_ctx* ctx, void* d_dst);
lbm_status lbm_set_state(lbm_ctx* ctx, const void* d_src, int64_t steps_done);

/* Kernel timing with HIP events recorded on the context's stream around each of the four
 * launches of every step (colour, extrap, normal, collide) while enabled. Enabling resets the
 * totals. lbm_kernel_times writes the accumulated device time in milliseconds of each of the
 * four kernels (host array of 4) and the number of timed steps. Timing does not change results.
 * Errors: LBM_ERR_HIP if an event cannot be created or queried. */
lbm_status lbm_set_profiling(lbm_ctx* ctx, int32_t enable);
lbm_status lbm_kernel_times(lbm_ctx* ctx, double* kernel_ms, int64_t* steps);

/* Discrete adjoint of the step, for gradients of the gas production L = m^p(T) - m^p(0)
 * (eqs. product_mass, production_rate) with respect to the per-node contact angle theta(x)
 * (eq. realigned_normal_vectors) and the reaction rate xi (eq. reactive_boundary_condition_*).
 * An adjoint state holds 30 planes of reals (context's real type) P elements apart (the plane
 * stride of lbm_state_layout), in the order of the state:
 * 19 colour-blind populations, the colour fraction a (dL/da; e moves with a, de/da = 1 on
 * either side of its sign), the three components of the recolouring vector v, 7 species
 * populations, each plane indexed by fluid id like the state (entries
 * f >= nfluid are zero). lbm_adjoint_bytes gives its size and the size of the scratch buffer
 * lbm_adjoint_step needs (both caller-owned device memory). */
lbm_status lbm_adjoint_bytes(const lbm_params* params, size_t* adj_bytes, size_t* scratch_bytes);

/* Size of a buffer for the forward fields of one level (rho^N, the realigned normal n* with
 * |grad rho^N|, the normal before realignment at wetting nodes, rho^m), for lbm_step_fields,
 * lbm_step_from and lbm_adjoint_step_fields. */
lbm_status lbm_fields_bytes(const lbm_params* params, size_t* bytes);

/* One time step, enqueued like lbm_step_async, that computes its level-t fields (the state
 * before the step) in d_fields (device memory of lbm_fields_bytes, caller-owned) instead of the
 * context's workspace. Same kernels and results as lbm_step. For checkpoint recomputation:
 * lbm_adjoint_step_fields then reuses the fields instead of recomputing them. */
lbm_status lbm_step_fields(lbm_ctx* ctx, void* d_fields);

/* One time step (the composite update of Sec. II: streaming, colour gradient and wetting,
 * forcing, central-moment collision, recolouring, wall reaction, species) from the state in
 * d_src to the state in d_dst, both caller-owned device buffers of lbm_state_bytes in the layout
 * of lbm_get_state. The context's own state and step count are left as they are; its geometry,
 * parameters and per-step workspace fields are used. d_fields: NULL, or a buffer of
 * lbm_fields_bytes that receives the level-t fields of d_src as lbm_step_fields writes them.
 * d_dst may be NULL when d_fields is not: then only the fields are computed (the colour,
 * extrapolation and normal passes; no collision, no state written), as a recomputation needs for
 * the last level of a segment. Enqueued only, like lbm_step_async: no reductions, no non-finite
 * report. Results are bitwise those of lbm_step from the same state. For checkpoint
 * recomputation that keeps every level without copying states. Errors: LBM_ERR_ARG for a NULL
 * source, for NULL d_dst and d_fields together, or overlapping buffers; LBM_ERR_HIP. */
lbm_status lbm_step_from(lbm_ctx* ctx, const void* d_src, void* d_dst, void* d_fields);

/* FP64 sums of the stored state d_state (lbm_state_bytes, as from lbm_get_state; NULL = the
 * context's current state), computed on the device: mass_r and mass_p are the colour masses of
 * its level (eqs. reactant_mass, product_mass: every stored population is pulled exactly once,
 * so the sum over the stored state equals the sum over the pulled level), species_total the
 * stored species total, nonfinite the count of fluid nodes holding a non-finite value;
 * conversion is 0 (it belongs to a step, not to a state). mass_p is the quantity whose
 * derivative lbm_adjoint_seed writes, so L = m^p(T) - m^p(0) of the adjoint is the difference
 * of two such calls. Uses the context's per-step partial sums (free between calls) and
 * synchronizes the stream. Errors: LBM_ERR_ARG for a NULL out, LBM_ERR_HIP. */
lbm_status lbm_state_sums(lbm_ctx* ctx, const void* d_state, lbm_reductions* out);

/* Writes dL/dS_T for L = m^p(T) into d_adj, given the state d_state (lbm_state_bytes, as from
 * lbm_get_state) of level T. Stream-ordered. */
lbm_status lbm_adjoint_seed(lbm_ctx* ctx, const void* d_state, void* d_adj);

/* One reverse step: given the state S_t (d_state, device, lbm_state_bytes) and
 * lambda_{t+1} = dL/dS_{t+1} (d_adj_in), writes lambda_t = dL/dS_t into d_adj_out (a different
 * buffer) and adds (dS_{t+1}/dtheta)^T lambda_{t+1} to d_grad_theta (device, N doubles, nonzero
 * only at wetting nodes) and (dS_{t+1}/dxi)^T lambda_{t+1} to *d_grad_xi (device, 1 double).
 * d_scratch: device memory of the scratch size from lbm_adjoint_bytes. Uses the context's
 * parameters and geometry and overwrites its per-step scratch fields (not its state). At the
 * non-smooth points of the step (minimum in the reaction cap, gradient and wetting-cone
 * guards) the derivative of the branch taken is used. With FP16/BF16 deviation storage the
 * adjoint is that of the FP32 arithmetic at the stored states, the storage rounding taken as the
 * identity (per-node contact-angle gradients are then usable in FP16 but not in BF16; integral
 * quantities such as dL/dxi hold in both). Stream-ordered; errors: LBM_ERR_ARG for a null
 * buffer or when a buffer the step writes (d_adj_out, d_scratch) overlaps another of its
 * buffers, LBM_ERR_HIP. */
lbm_status lbm_adjoint_step(lbm_ctx* ctx, const void* d_state, const void* d_adj_in, void* d_adj_out,
                            void* d_scratch, double* d_grad_theta, double* d_grad_xi);

/* lbm_adjoint_step with the level-t fields of d_state taken from d_fields (as written by
 * lbm_step_fields from the same state) instead of recomputed; otherwise identical, bit for
 * bit. Errors as lbm_adjoint_step. */
lbm_status lbm_adjoint_step_fields(lbm_ctx* ctx, const void* d_state, const void* d_fields, const void* d_adj_in,
                                   void* d_adj_out, void* d_scratch, double* d_grad_theta, double* d_grad_xi);

/* Number of steps taken since init (or the value given to lbm_set_state). */
int64_t lbm_steps_done(const lbm_ctx* ctx);

/* Releases the context (host memory only; the workspace belongs to the caller). */
void lbm_free(lbm_ctx* ctx);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): lbm_adjoint_step without the d_scratch argument. Its
 * scratch is a fixed array of lbm_adjoint_static_scratch_bytes() (64 MiB) inside the library,
 * one per device, held until the process ends; the call allocates nothing. Same arguments,
 * results (bit for bit) and errors as lbm_adjoint_step, plus LBM_ERR_ARG when the problem needs
 * more scratch than the array holds (lbm_adjoint_bytes reports the need: about 8 r N + 12 r F
 * bytes for N nodes, F fluid nodes, r = 4 in FP32/FP16/BF16 and 8 in FP64; the 96^3 porous
 * workload fits in FP32, not in FP64) and LBM_ERR_HIP if the array's device address cannot be
 * resolved. Every call on one device shares that device's array and leaves its contents behind:
 * calls that overlap in time on one device (two streams, two threads) race and must be ordered
 * by the caller; every value a call reads from the array it has written first. */
lbm_status lbm_adjoint_step_static(lbm_ctx* ctx, const void* d_state, const void* d_adj_in, void* d_adj_out,
                                   double* d_grad_theta, double* d_grad_xi);
size_t lbm_adjoint_static_scratch_bytes(void);

/* Message of the last error on this context (context-owned storage), or with ctx NULL of the
 * last failed call without a context on the calling thread (thread-local storage); never NULL. */
const char* lbm_last_error(const lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
