/*
 * lbm.h -- C ABI of the MI355X (gfx950) implementation of the vectorial
 * lattice Boltzmann method for 2D linear elastodynamics
 * (Boolakee, Geier, De Lorenzis, arXiv 2408.01081).
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - C linkage, plain pointers and sizes; every function returns lbm_status
 *    and never throws.  On error the context is left unchanged and
 *    lbm_last_error() returns a thread-local message.
 *  - "d_" pointers are device memory on the device that was current when the
 *    context was created; "h_" pointers are host memory.
 *  - The caller owns all device memory.  The library never allocates device
 *    memory: the workspace passed to lbm_create holds the whole lattice state
 *    and must outlive the context.  Input arrays must stay valid until the
 *    stream has consumed them.
 *  - All device work is enqueued on the HIP stream given at creation
 *    (NULL = the null stream) and is asynchronous, except the calls that
 *    return host scalars (lbm_energy, lbm_rel_l2), which synchronise the
 *    stream.
 *  - Field arrays are row-major [component][ny][nx] with x fastest.  Node
 *    (k,l) sits at ((k+1/2)dx, (l+1/2)dx); for Dirichlet problems the walls
 *    are the lines x = 0, x = nx dx, y = 0, y = ny dx, half a spacing outside
 *    the outermost nodes (q_ij = 1/2, Eq. bc_q).
 *  - Units are the caller's (physical).  Internally the scheme runs on the
 *    first-order system's variables U = (v_x, v_y, j_s, j_d, j_xy)
 *    (Eq. system) with populations in FP32.
 *  - One context must not be used from two host threads at once.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
  LBM_OK = 0,
  LBM_E_ARG = 1,   /* invalid argument (null pointer, size, range)          */
  LBM_E_CFL = 2,   /* 2 sqrt(c_K^2 + c_mu^2) >= dx/dt (Eq. stab_cond)        */
  LBM_E_STATE = 3, /* call out of order (e.g. step before init)              */
  LBM_E_SPACE = 4, /* workspace too small                                    */
  LBM_E_HIP = 5    /* a HIP runtime call failed; see lbm_last_error()         */
} lbm_status;

typedef enum { LBM_PERIODIC = 0, LBM_DIRICHLET = 1 } lbm_bc;

/* How lambda is read (Section 2.1, Eqs. 2D / plane_strain / plane_stress):
 *   LBM_PLANE_STRAIN  lambda is the 3D Lame constant: c_K^2 = (lambda+mu)/rho
 *   LBM_CONTINUUM_2D  lambda is the 2D Lame constant: c_K^2 = (lambda+mu)/rho
 *   LBM_PLANE_STRESS  c_K^2 = (lambda* + mu)/rho, lambda* = 2 lambda mu/(lambda+2mu)
 * In all cases c_mu^2 = mu/rho (Eq. all). */
typedef enum { LBM_PLANE_STRAIN = 0, LBM_PLANE_STRESS = 1, LBM_CONTINUUM_2D = 2 } lbm_model;

typedef struct {
  int32_t nx, ny;      /* nodes per side, >= 1, nx * ny <= 2^31                   */
  double dx, dt;       /* lattice spacing and time step; c = dx/dt               */
  double lambda, mu;   /* Lame constants; mu >= 0, lambda + mu > 0 (mu = 0: see
                          lbm_init_from_gradient; batched instances need mu > 0) */
  double rho;          /* density > 0                                            */
  int32_t bc;          /* lbm_bc                                                 */
  int32_t model;       /* lbm_model                                              */
  uint32_t flags;      /* 0 or LBM_F_PLANE_LAYOUT | LBM_F_DISPLACEMENT | ...      */
} lbm_params;

/* Population layout in the workspace (both: 20 FP32 planes, x fastest, rows
 * padded to 64 floats).  Default: row-major [y][plane][x], the 20 plane rows
 * of one lattice row contiguous.  LBM_F_PLANE_LAYOUT: plane-major
 * [plane][y][x].  Results are bitwise identical; only speed differs. */
#define LBM_F_PLANE_LAYOUT 1u

/* LBM_F_DISPLACEMENT: the workspace also holds a displacement state
 * [2][ny][nx] FP32, integrated by the trapezoidal rule (Section 3.5) inside
 * every step (16 B per node); see lbm_init_displacement.  Single lattices
 * only. */
#define LBM_F_DISPLACEMENT 2u

/* LBM_F_ALLOW_UNSTABLE: accept parameters that violate the CFL-like
 * condition Eq. stab_cond, to reproduce the divergence of the unstable pair
 * of Section 6.2.  Above the limit some g_ij is not positive definite and the
 * weighted norm does not exist: lbm_energy then returns the plain sum of
 * squares of the populations.  Single lattices only. */
#define LBM_F_ALLOW_UNSTABLE 4u

/* Device bytes the workspace must provide for these parameters (0 if the
 * parameters are invalid). */
size_t lbm_workspace_bytes(const lbm_params* p);

/* Validate parameters (including the CFL-like condition, Eq. stab_cond),
 * derive the Courant numbers kK = c_K dt/dx, km = c_mu dt/dx and the norm
 * weights k_ij = g_ij^{-1} (Eq. def_symmetrizer), bind the workspace and the
 * stream.  *out receives a host-allocated context (free with lbm_destroy).
 * d_ws must be 256-byte aligned. */
lbm_status lbm_create(const lbm_params* p, void* d_ws, size_t ws_bytes, void* hip_stream,
                      lbm_ctx** out);

/* Second-order initialisation (Eq. ic_second) from physical initial data,
 * computed in FP64 and rounded once to FP32, at time t = 0.
 *   d_v0      [2][ny][nx] FP64  initial velocity v0 = d_t u0 (Eq. init_v)
 *   d_sigma0  [3][ny][nx] FP64  initial Cauchy stress (xx, yy, xy) of u0
 *   d_grad    nullable [2][5][ny][nx] FP64: d/dx then d/dy of
 *             (v_x, v_y, sigma_xx, sigma_yy, sigma_xy) at the nodes; when
 *             NULL the library uses second-order central differences
 *             (periodic wrap; one-sided second order at Dirichlet walls).
 * The stress is converted to U through Eq. sigma_num:
 *   j_s = -(s_xx+s_yy)/(2 c_K), j_d = -(s_xx-s_yy)/(2 c_mu), j_xy = -s_xy/c_mu,
 * s = sigma/rho.  Resets the step counter to 0. */
lbm_status lbm_init(lbm_ctx* ctx, const double* d_v0, const double* d_sigma0,
                    const double* d_grad);

/* The same initialisation (Eq. ic_second) from the initial velocity and the
 * gradient of the initial displacement, through Eq. ic_vector:
 *   U0 = (v0x, v0y, -c_K (du_x/dx + du_y/dy), -c_mu (du_x/dx - du_y/dy),
 *         -c_mu (du_y/dx + du_x/dy)),
 * which involves no division by c_mu: the entry point for mu = 0 (c_mu = 0,
 * the (c_K^2, c_mu^2) = (1.5, 0) material of Section 6.1), where lbm_init
 * fails with LBM_E_ARG.
 *   d_v0      [2][ny][nx] FP64  initial velocity
 *   d_gradu0  [4][ny][nx] FP64  du_x/dx, du_x/dy, du_y/dx, du_y/dy of u0
 *   d_grad    nullable [2][6][ny][nx] FP64: d/dx then d/dy of the six input
 *             fields (v_x, v_y, du_x/dx, du_x/dy, du_y/dx, du_y/dy), physical
 *             units; when NULL the library takes second-order central
 *             differences of U0 (periodic wrap; one-sided second order at
 *             Dirichlet walls).
 * Computed in FP64, rounded once to FP32; resets the step counter to 0. */
lbm_status lbm_init_from_gradient(lbm_ctx* ctx, const double* d_v0, const double* d_gradu0,
                                  const double* d_grad);

/* Load FP32 populations directly ([4][5][ny][nx], pre-collision, directions
 * in the paper's order (1,0),(0,1),(-1,0),(0,-1), components of U) at step
 * counter 0, collided with the body load of t_0 (if one is set; Eq. cond_eq).
 * For checkpoints and parity tests;
 * a context with LBM_F_DISPLACEMENT still needs lbm_init_displacement. */
lbm_status lbm_set_populations(lbm_ctx* ctx, const float* d_f);

/* Time-dependent Dirichlet data (Eq. bc_ansatz with source Eq. bc_s) in
 * separable form: the wall velocity du_D/dt at the midpoint x_b of wall link
 * L at time t_n + dt/2 is  sum_r d_W[r][L][0..1] * d_T[n][r].
 *   rank   R >= 0 (0 = homogeneous walls; pointers may then be NULL)
 *   d_W    [R][2(nx+ny)][2] FP32, link order: left wall (node (0,l), l-major),
 *          right wall (node (nx-1,l)), bottom wall (node (k,0)),
 *          top wall (node (k,ny-1))
 *   d_T    [nsteps][R] FP32, row n = time functions at t_n + dt/2
 * Steps beyond nsteps are rejected by lbm_step.  The source rows 3-5 use
 * c_K/c and c_mu/c (the leading-order bounce-back balance, Eq. bb0, carries
 * the 1/c of the equilibrium; the printed speeds coincide only for c = 1).
 * lbm_step sums the series for chunks of up to 420 steps into a table inside
 * the workspace (one small launch per chunk, FMA in rank order), so the step
 * kernels read one velocity per wall link.  Pointers are kept (not copied)
 * and must stay valid while stepping. */
lbm_status lbm_set_wall_velocity(lbm_ctx* ctx, int32_t rank, const float* d_W,
                                 const float* d_T, int64_t nsteps);

/* Body load b_bar = rho b (Eq. cond_eq: B_hat = dt b_bar / rho) in separable
 * form: at node (k, l) and time level t_n
 *   b_bar_a(x_k, y_l, t_n) = sum_r d_X[r][a][k] * d_Y[r][l] * d_T[n][r],
 * a = x, y component (a product of a function of x, a function of y and a
 * function of t per term, e.g. the expansion of sin(a x + b y + w t)).
 *   rank   R in 0..4096 (0 = no load; pointers may then be NULL)
 *   d_X    [R][2][nx] FP32,  d_Y  [R][ny] FP32,
 *   d_T    [nsteps + 1][R] FP32, row n = time functions at t_n
 * The load enters the initialisation (Eq. ic_second), the collision
 * (U_num = sum f + B_hat / 2 at every collision) and every output at the
 * current level.  Steps beyond nsteps are rejected by lbm_step.  With a
 * blocked variant selected (lbm_set_tblock_config / lbm_autotune), R <= 32,
 * no error tracking and ny >= T + 5, steps run T per launch of a blocked
 * kernel with the load (and the displacement state if the context keeps
 * it), bitwise the same results, and the steps after the last full launch
 * in as few launches of shorter blocked variants as exist (a last single
 * step in the one-node-per-thread kernel); otherwise one launch per step of
 * the one-node-per-thread kernel (lbm_steps_per_launch tells which).  Set it
 * before lbm_init to include B_hat(0) in the initialisation.  Pointers are
 * kept (not copied) and must stay valid while stepping. */
lbm_status lbm_set_body_force(lbm_ctx* ctx, int32_t rank, const float* d_X, const float* d_Y,
                              const float* d_T, int64_t nsteps);

/* Start the displacement output (Section 3.5, Eq. trapezoidal: u(t_{n+1}) =
 * u(t_n) + dt/2 (v(t_n) + v(t_{n+1}))) from u0 = d_u0 [2][ny][nx] FP64, right
 * after lbm_init (step counter 0).  The workspace keeps D = u + dt/2 v_num
 * in FP64 (a running sum: FP32 would round the whole displacement at every
 * half step); each step adds dt/2 v_num twice.  Requires LBM_F_DISPLACEMENT;
 * lbm_step rejects a context with the flag until this has been called.
 * With a blocked variant selected (and a body load of rank <= 32 or none,
 * no error tracking) steps run several per launch, the rows in flight kept
 * in LDS and updated in the same order (bitwise the same D); otherwise one
 * launch per step. */
lbm_status lbm_init_displacement(lbm_ctx* ctx, const double* d_u0);

/* Displacement u(t_n) = D - dt/2 v_num(t_n) at the current step, [2][ny][nx]
 * FP32 (x then y component). */
lbm_status lbm_displacement(lbm_ctx* ctx, float* d_u);

/* ---- error norms against an exact solution (Section 6.1) ------------------
 * The exact outputs in separable form, FP64: at node (k, l) and level t_n
 *   phi_c(x_k, y_l, t_n) = sum_r d_X[r][c][k] * d_Y[r][l] * d_T[n][r],
 * c = u_x, u_y, v_x, v_y, sigma_xx, sigma_yy, sigma_xy (Cauchy stress).
 *   rank   R in 0..4096 (0 removes the reference and stops tracking)
 *   d_X    [R][7][nx],  d_Y  [R][ny],  d_T  [nsteps + 1][R]
 * Pointers are kept (not copied) and must stay valid while tracking. */
lbm_status lbm_set_reference(lbm_ctx* ctx, int32_t rank, const double* d_X, const double* d_Y,
                             const double* d_T, int64_t nsteps);

/* on != 0: zero the running sums, add the current level, and from then on
 * add every level lbm_step forms (steps then run one launch per step);
 * on == 0: stop adding.  lbm_init and lbm_set_populations stop tracking.
 * Per level and node the numerical outputs are formed as lbm_moments and
 * lbm_displacement form them (the displacement group needs
 * LBM_F_DISPLACEMENT and lbm_init_displacement, else it stays zero) and the
 * differences to phi are summed in FP64 with fixed-order reductions. */
lbm_status lbm_error_track(lbm_ctx* ctx, int32_t on);

/* Running sums since tracking started, h_out[10] FP64: for the groups
 * u (u_x, u_y), v (v_x, v_y) and sigma (3 components), in that order,
 * sum over levels and nodes of |e|^2, of |phi|^2 and the maximum of
 * |e|_inf; then the number of levels added.  The norms of Section 6.1
 * follow as L2(e) = (dx^2 dt sum |e|^2)^(1/2), L2rel = (sum |e|^2 /
 * sum |phi|^2)^(1/2), Linfrel = max |e|_inf / L2(phi).  Synchronises. */
lbm_status lbm_error_sums(lbm_ctx* ctx, double* h_out);

/* Advance n >= 0 time steps (Section 3.6: collision with omega = 2, then
 * streaming with periodic wrap or the Dirichlet rule), asynchronously. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n);

/* Steps taken since lbm_init / lbm_set_populations. */
int64_t lbm_step_count(const lbm_ctx* ctx);

/* Macroscopic output at the current step (Section 3.5):
 *   d_out  [5][ny][nx] FP32: v_x, v_y, sigma_xx, sigma_yy, sigma_xy (Cauchy,
 *          Eq. sigma_num times rho). */
lbm_status lbm_moments(lbm_ctx* ctx, float* d_out);

/* The first-order system's variables U_num = sum_ij f_ij + dt/2 B
 * (Eq. cond_eq) at the current step, [5][ny][nx] FP32. */
lbm_status lbm_moments_U(lbm_ctx* ctx, float* d_U);

/* Pre-collision populations at the current step, [4][5][ny][nx] FP32. */
lbm_status lbm_populations(lbm_ctx* ctx, float* d_f);

/* Squared weighted L2 grid norm ||f||_P^2 = sum_x sum_ij f_ij^T k_ij f_ij
 * (Definition grid_norm, Eq. def_symmetrizer), accumulated in FP64.
 * Synchronises the stream. */
lbm_status lbm_energy(lbm_ctx* ctx, double* h_out);

/* Relative L2 difference ||U_num - U_ref|| / ||U_ref|| over all nodes and the
 * five components of U, accumulated in FP64; d_ref is [5][ny][nx] FP64 in the
 * first-order system's variables.  Synchronises the stream. */
lbm_status lbm_rel_l2(lbm_ctx* ctx, const double* d_ref, double* h_out);

/* Courant numbers (kK, kmu) and lattice speed c of a context. */
lbm_status lbm_lattice_constants(const lbm_ctx* ctx, double* h_kK, double* h_kmu, double* h_c);

/* ---- launch configurations of the step kernel and the autotuner ----------
 * Every configuration performs the same per-node FP32 arithmetic, so all
 * give bitwise-identical results; they differ in nodes per thread (vector
 * width of the accesses), threads per workgroup, nontemporal stores and how
 * the x-shifted neighbour values are obtained (extra load or lane shuffle).
 * A configuration is valid for a grid when nx is a multiple of its vector
 * width (and of 64 x width for the lane-shuffle variants). */
int32_t lbm_step_config_count(void);
lbm_status lbm_step_config_info(int32_t index, int32_t* h_vec, int32_t* h_threads,
                                int32_t* h_nontemporal, int32_t* h_shuffle);
lbm_status lbm_get_step_config(const lbm_ctx* ctx, int32_t* h_index);
lbm_status lbm_set_step_config(lbm_ctx* ctx, int32_t index);

/* Time every valid configuration on this context's grid (reps launches each
 * after two warm-up launches, HIP events on the context's stream), including
 * the temporally blocked variants below (compared per step), and select the
 * fastest single-step configuration (*h_index) and, when it is faster per
 * step, a blocked variant (read it with lbm_get_tblock_config).  Launches are
 * timed with the context's wall data at the current step when it has data for
 * seven more steps, else with resting walls.  The lattice state is not
 * modified: timed launches read the current state and write the spare buffer.
 * With use_cache != 0 a previous result for the same (nx, ny, bc) in this
 * process, or in the file named by the environment variable
 * LBM_AUTOTUNE_CACHE, is reused without timing (*h_ms = -1 then).  New
 * results (the selected variants, and those for the last steps of a run) are
 * appended to that file.  *h_ms = best time per step.
 * Synchronises. */
lbm_status lbm_autotune(lbm_ctx* ctx, int32_t reps, int32_t use_cache, int32_t* h_index,
                        double* h_ms);

/* ---- several time steps per launch (temporal blocking) ----------------------
 * The scheme's update of a node needs only its four neighbours (pull
 * streaming, Eq. streaming, then the local collision, Eq. collision), so T
 * consecutive steps of a row need rows within distance T of the previous
 * state.  A wave owns a strip of 64 columns and sweeps a segment of rows,
 * forming the T - 1 intermediate time levels in registers, so T steps read and
 * write the populations once (80 B + 80 B per node for T updates).  Bitwise
 * identical to T single steps.  Variants (h_steps = T in 2..10) differ in rows
 * per segment, store type and rows prefetched ahead (h_prefetch); h_seg_rows
 * 0 means the segment length is chosen at launch so that one wave per
 * resident slot covers the grid, -k that k waves per slot do, -100 that one
 * wave per SIMD (4 per CU) does whatever the occupancy.  index -1 disables blocking; lbm_autotune
 * selects a variant when it is faster per step than the best single-step
 * configuration.  With a variant of T steps enabled, lbm_step(n) runs the
 * steps in chunks of floor(420 / T) T steps, T per launch; the r = n mod T
 * steps after the last full launch take one launch of an r-step variant
 * (the fastest one lbm_autotune timed, else the r-step variant of the
 * nearest launch shape), or of the single-step kernel for r = 1.  Row base
 * addresses are 64-bit; only the byte offsets inside one row's 20 planes
 * ((19 plane strides + one row) * 4 B) must stay below 2^31, which fails
 * for the plane-major layout beyond about 28 M nodes and for rows of more
 * than about 13 M nodes: setting or timing a variant then fails with
 * LBM_E_ARG and the autotuner skips it.  Any output pointer may be NULL. */
int32_t lbm_tblock_config_count(void);
lbm_status lbm_tblock_config_info(int32_t index, int32_t* h_steps, int32_t* h_seg_rows,
                                  int32_t* h_nontemporal, int32_t* h_prefetch);
/* Time steps per launch that lbm_step uses for this context as configured
 * now: T of the selected blocked variant (with a body load and/or the
 * displacement state: of the variant with those extras that lbm_step picks
 * for it), 1 for single steps or while error norms are tracked; -1 for a
 * NULL context. */
int32_t lbm_steps_per_launch(const lbm_ctx* ctx);
lbm_status lbm_get_tblock_config(const lbm_ctx* ctx, int32_t* h_index);
lbm_status lbm_set_tblock_config(lbm_ctx* ctx, int32_t index);
/* Split blocked launches of a Dirichlet lattice (Eq. bc_ansatz acts only at
 * the walls and a step moves information one node, so after T steps the
 * nodes at least T from every wall hold what periodic arithmetic on the same
 * rows gives: bitwise the same operations).  A split launch sweeps the
 * interior (the strips whose stored columns lie in [T, nx - T), rows
 * 16 .. ny - 17) with the periodic kernel's code, which keeps the wall
 * code's registers out of it, and the band along the walls with the
 * Dirichlet rule as 16-row segments, in one grid; results are bitwise those
 * of the unsplit launch.  Variants with T, store type and prefetch of a
 * split kernel (T = 7, 6 with one or two rows prefetched, T = 5 with one;
 * plain stores; at T = 8 the Dirichlet code keeps scratch spills and no
 * split kernel is built) run split where the lattice allows it (at least
 * one interior strip, and ny >= 33).  mode -1 (default) or 1: split those;
 * 0: never.  LBM_E_ARG for another mode.  The autotuner's choices are kept
 * per mode. */
lbm_status lbm_set_tblock_split(lbm_ctx* ctx, int32_t mode);
/* 1 if launches of blocked variant `index` run split on this context as
 * configured now, 0 if not, -1 for a NULL context or a bad index. */
int32_t lbm_tblock_split_active(lbm_ctx* ctx, int32_t index);
/* Select the launch configuration that makes runs of nsteps steps cheapest:
 * for every blocked variant (and for single steps) the predicted time of such
 * a run from the launch times the last lbm_autotune of this shape in this
 * process measured, floor(nsteps / T) full launches plus the launch lbm_step
 * takes for the nsteps mod T steps left; the cheapest becomes the selected
 * variant (*h_index, -1: single steps).  A variant that divides nsteps can
 * win over one that is faster per step (4096^2: T = 10 for 20-step runs,
 * against T = 8 per step).  Without such launch times (no lbm_autotune, or
 * its choice read from the cache file) the selection is unchanged.
 * Applies to lbm_step without a body load, displacement state or error
 * tracking.  LBM_E_ARG for a NULL argument or nsteps < 1. */
lbm_status lbm_select_for_steps(lbm_ctx* ctx, int64_t nsteps, int32_t* h_index);
/* The r-step blocked variant (r = 2 .. 10) lbm_step launches for the last r
 * steps of a run when r is below the selected variant's T: the fastest
 * r-step variant lbm_autotune timed (kept in its cache file as well), else
 * the r-step variant nearest to the selected one's launch shape;
 * *h_index = -1 when no variant is selected or r is outside 2 .. 10.
 * LBM_E_ARG for a NULL argument. */
lbm_status lbm_get_tblock_remainder(const lbm_ctx* ctx, int32_t r, int32_t* h_index);
/* Average duration (ms) of one launch of blocked variant `index` (T steps;
 * state-preserving, synchronises). */
lbm_status lbm_time_tblock_config(lbm_ctx* ctx, int32_t index, int32_t reps, double* h_ms);

/* Average duration (ms) of one step launch of configuration `index` on this
 * context (same state-preserving scheme as lbm_autotune).  Synchronises. */
lbm_status lbm_time_step_config(lbm_ctx* ctx, int32_t index, int32_t reps, double* h_ms);

/* Plain streaming copy of n floats (n % 4 == 0, 16-byte aligned buffers) on
 * the given stream: the bandwidth and memory-counter reference kernel. */
lbm_status lbm_copy_f32(float* d_dst, const float* d_src, int64_t n, void* hip_stream);

/* ---- the exact linear window operator of a periodic lattice -------------------
 * On a periodic lattice with a fixed material the map from fields to the
 * fields 16 steps later, through the second-order initialisation with
 * central-difference gradients (Eq. ic_second), 16 steps (Section 3.6) and
 * the outputs of Section 3.5, is linear (Eq. collision_vector and
 * Eq. streaming are linear) and commutes with lattice shifts: a convolution
 * whose taps are the responses to unit deltas, zero outside the diamond
 * |dx| + |dy| <= 17 (one node per step, one more for the central
 * differences).  The same map as lbm_init + lbm_step(16) + lbm_moments on
 * such a lattice, in one launch, up to FP32 rounding. */
#define LBM_WOP_STEPS 16
#define LBM_WOP_SIDE 35               /* taps per side: 2 (16 + 1) + 1 */
#define LBM_WOP_OPERAND_BYTES 262144  /* packed operator for lbm_wop_apply */

/* Device scratch lbm_wop_build needs for these parameters (0 if invalid:
 * Dirichlet, mu = 0, or failing lbm_create's checks).  Only the material,
 * dx and dt of p matter for the build; nx and ny are ignored. */
size_t lbm_wop_scratch_bytes(const lbm_params* p);
size_t lbm_wop_operand_bytes(void);

/* Build the operator for p's material and time step: unit deltas in each
 * component of U go through the library's own FP64 initialisation and 16
 * FP32 steps on a 40 x 40 periodic lattice set up on d_scratch
 * (lbm_wop_scratch_bytes, 256-byte aligned).
 *   d_G   nullable [35][35][5][5] FP32: G[dy + 17][dx + 17][co][ci], the
 *         response in U_co at offset (dx, dy) to a unit delta in U_ci
 *   d_op  LBM_WOP_OPERAND_BYTES, 16-byte aligned: the taps in the physical
 *         fields (v, sigma_bar), packed for lbm_wop_apply
 * Requires a periodic problem with mu > 0 (LBM_E_ARG otherwise).  Enqueued
 * on hip_stream; the scratch must stay valid until the stream has run it. */
lbm_status lbm_wop_build(const lbm_params* p, float* d_G, void* d_op, void* d_scratch,
                         size_t scratch_bytes, void* hip_stream);

/* Apply the operator to `batch` periodic windows of p->nx x p->ny (any sizes
 * >= 1; p->bc periodic): d_in, d_out [batch][5][ny][nx] FP32 physical fields
 * (v_x, v_y, sigma_xx, sigma_yy, sigma_xy), not overlapping.  One launch of
 * FP32 matrix-core products (v_mfma_f32_16x16x4_f32) with the input tile of
 * each workgroup staged in LDS. */
lbm_status lbm_wop_apply(const lbm_params* p, const void* d_op, const float* d_in, float* d_out,
                         int32_t batch, void* hip_stream);

/* ---- batched lattices --------------------------------------------------------
 * n independent instances, each with its own lbm_params (size, boundary,
 * material, dx, dt; flags must be 0), advanced together: one launch per time
 * step (or per T steps, below) covers every instance, with the same per-node
 * arithmetic as lbm_step (results are bitwise identical to stepping each
 * instance alone).  lbm_batch_step(n) executes the launches as one hipGraph
 * (built node by node and cached per step count, buffer parity and blocked
 * variant while no instance has wall data).  The caller owns the workspace;
 * the library never allocates device memory.
 *
 * Packed field arrays hold instance i's fields contiguously as
 * [component][ny_i][nx_i], starting at (component count) x
 * lbm_batch_node_offset(b, i); lbm_batch_node_offset(b, n) is the total number
 * of nodes. */
typedef struct lbm_batch lbm_batch;

size_t lbm_batch_workspace_bytes(int32_t n, const lbm_params* h_params);
lbm_status lbm_batch_create(int32_t n, const lbm_params* h_params, void* d_ws, size_t ws_bytes,
                            void* hip_stream, lbm_batch** out);
int64_t lbm_batch_node_offset(const lbm_batch* b, int32_t i);
int64_t lbm_batch_step_count(const lbm_batch* b);

/* FP64 second-order initialisation (Eq. ic_second, central-difference
 * gradients) of every instance from packed physical fields:
 * d_v0 [..][2][ny][nx], d_sigma0 [..][3][ny][nx] (Cauchy stress), FP64. */
lbm_status lbm_batch_init(lbm_batch* b, const double* d_v0, const double* d_sigma0);

/* Same, from one packed FP32 array [..][5][ny][nx] = (v_x, v_y, sigma_xx,
 * sigma_yy, sigma_xy) per instance (the layout lbm_batch_moments writes);
 * computed in FP64. */
lbm_status lbm_batch_init_fields_f32(lbm_batch* b, const float* d_fields);

/* Wall data of Dirichlet instance i, as lbm_set_wall_velocity. */
lbm_status lbm_batch_set_wall_velocity(lbm_batch* b, int32_t i, int32_t rank, const float* d_W,
                                       const float* d_T, int64_t nsteps);

/* Advance every instance n steps: one hipGraph launch of the step kernels
 * (one step per kernel, or T per kernel with a blocked variant selected; the
 * r = n mod T steps after the last full launch as one launch of an r-step
 * variant for r >= 2 -- the fastest one lbm_batch_autotune timed, else the
 * one nearest to the selected variant's shape -- or one step for r = 1). */
lbm_status lbm_batch_step(lbm_batch* b, int64_t n);

/* Same steps launched one kernel at a time (no graph). */
lbm_status lbm_batch_step_eager(lbm_batch* b, int64_t n);

/* Temporally blocked batched steps: the blocked sweep of lbm_tblock_config_*
 * applied to every instance in one launch per T steps (a table maps each wave
 * to its instance, strip and segment); bitwise identical to single steps.
 * Instances with wall data (lbm_batch_set_wall_velocity with rank > 0): a
 * small launch before each blocked launch sums the wall velocities of its T
 * steps into a per-instance table in the workspace (as lbm_set_wall_velocity
 * data are summed for a single lattice), which the blocked kernel reads.
 * Index -1 = single steps.  Every variant's wave table is uploaded into the
 * workspace at lbm_batch_create; selecting a variant launches nothing.
 * lbm_batch_autotune times the single-step kernel and every usable variant on
 * the live state without changing it (reps launches each, HIP events), keeps
 * the launch times (they pick the launch for the last steps of a run),
 * selects the fastest per step and returns its index and ms per step; it
 * synchronises. */
int32_t lbm_batch_tblock_config_count(void);
lbm_status lbm_batch_tblock_config_info(int32_t index, int32_t* h_steps, int32_t* h_seg_rows,
                                        int32_t* h_nontemporal, int32_t* h_prefetch);
lbm_status lbm_batch_get_tblock_config(const lbm_batch* b, int32_t* h_index);
lbm_status lbm_batch_set_tblock_config(lbm_batch* b, int32_t index);
lbm_status lbm_batch_autotune(lbm_batch* b, int32_t reps, int32_t* h_index, double* h_ms);

/* Packed FP32 moments: (v, sigma_bar) or the system variables U, [..][5][ny][nx]. */
lbm_status lbm_batch_moments(lbm_batch* b, float* d_out);
lbm_status lbm_batch_moments_U(lbm_batch* b, float* d_U);

/* Per-instance ||f||_P^2 (FP64, fixed-order reduction) into h_out[n].  Synchronises. */
lbm_status lbm_batch_energy(lbm_batch* b, double* h_out);

/* Per-instance relative L2 difference between the current state and packed
 * FP32 physical fields [..][5][ny][nx] (v, sigma_bar), measured on the system
 * variables U: ||U - U(fields)|| / ||U|| (FP64) into h_out[n].  Synchronises. */
lbm_status lbm_batch_rel_l2_fields(lbm_batch* b, const float* d_fields, double* h_out);

/* Per-instance relative L2 difference between two packed FP32 physical field
 * arrays d_a, d_b [..][5][ny][nx] (v, sigma_bar), measured on the system
 * variables U of each instance's material (inverse of Eq. sigma_num, FP64):
 * ||U(a) - U(b)|| / ||U(b)|| into h_out[n].  Uses the batch's layout and
 * materials only (no lattice state; callable before any initialisation).
 * Synchronises. */
lbm_status lbm_batch_rel_l2_pair(lbm_batch* b, const float* d_a, const float* d_b,
                                 double* h_out);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving or evaluation loops and harnesses that
 * forbid it): lbm_batch_rel_l2_pair without a batch or workspace.  n
 * instances described by h_params (same rules as lbm_batch_create; the
 * fields are packed as for a batch of them), d_a and d_b as for
 * lbm_batch_rel_l2_pair; the same kernels and summation order, so the same
 * results.  Instance descriptors, tile table and partial sums go to a fixed
 * 4 MiB array of device memory inside the library, one per GPU, held until
 * the process ends (found with hipGetSymbolAddress on the first call on each
 * device, with that device current).  Limits: 1 <= n <= 256 (else
 * LBM_E_ARG) and at most 131072 row tiles, sum over instances of
 * ny * ceil(nx / 256) (else LBM_E_SPACE).  Calls no hipMalloc or hipFree.
 * All calls on one GPU share the array: calls that overlap on one GPU (from
 * other host threads, or on other streams) race.  Enqueued on hip_stream
 * (a stream of the current device); synchronises it. */
lbm_status lbm_rel_l2_pair_static(int32_t n, const lbm_params* h_params, const float* d_a,
                                  const float* d_b, double* h_out, void* hip_stream);

lbm_status lbm_batch_destroy(lbm_batch* b);

/* Release the host context (the workspace stays with the caller). */
lbm_status lbm_destroy(lbm_ctx* ctx);

/* Message describing the last error on this thread ("" if none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
