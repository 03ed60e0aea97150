/*
 * elb.h — C ABI of the MI355X finite-difference lattice Boltzmann (FDLB) solver for the
 * simplified Enskog equation with a Shakhov collision term (Busuioc, arXiv 2211.16933).
 *
 * One context advances one 1-D problem on nx cells with Q Gauss-Hermite momentum nodes
 * (Sec. II.D).  The state is the pair of reduced distributions phi_k, theta_k per cell
 * (Sec. II.C), stored quadrature-weighted (n = sum_k phi_k).  A time step is one pass of
 * the third-order TVD Runge-Kutta scheme (App. A.1, eq. rk3) over the right-hand side
 *   L_k = -(F_{i+1/2,k} - F_{i-1/2,k})/dx - (psi_k - psi_{S;k})/tau + J1_k
 * with WENO-5 fluxes (App. A.2), the Shakhov target built on the Hermite-expanded
 * equilibrium (Sec. II.C-D) and the simplified-Enskog source (eq. j1_expanded) whose
 * gradients are sixth-order central differences (App. A.3).
 *
 * Units: m = k_B = 1, T_ref = 1 (Sec. II.A).
 *
 * Conventions for every entry point:
 *  - Every call returns an elb_status; on failure elb_last_error() describes it.
 *  - Host arrays are caller-owned and copied before the call returns.
 *  - Device memory is caller-owned: the caller allocates elb_workspace_bytes() bytes of
 *    device memory (256-byte aligned) and passes it to elb_create; the library keeps no
 *    other device allocation.  The workspace must outlive the context.
 *  - Work is enqueued on the HIP stream given to elb_create (NULL = default stream).
 *    elb_step is asynchronous; calls that return host data synchronise that stream.
 *  - A context is used from one host thread at a time.  Distinct contexts are
 *    independent.
 */
#ifndef ELB_H
#define ELB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct elb_ctx elb_ctx;

typedef enum {
    ELB_OK = 0,
    ELB_EINVAL = 1,        /* invalid parameter or input; nothing was launched          */
    ELB_ENOMEM = 2,        /* workspace too small or host allocation failed             */
    ELB_EHIP = 3,          /* HIP runtime error (message in elb_last_error)             */
    ELB_ENONFINITE = 4,    /* a cell reached n <= 0, T <= 0 or a non-finite moment      */
    ELB_ESTATE = 5,        /* call out of order (e.g. step before a state is set)       */
    ELB_EUNSUPPORTED = 6   /* valid request the library does not implement (e.g. a Q)   */
} elb_status;

enum { ELB_BC_PERIODIC = 0, ELB_BC_EQUILIBRIUM = 1 };
enum { ELB_PR_CONST = 0, ELB_PR_ENSKOG = 1 };
enum { ELB_FP64 = 0, ELB_FP32 = 1, ELB_FP32_MIXED = 2 };
enum { ELB_CHI_SET = 0, ELB_CHI_RETFM = 1 };

/* Problem description (zero-initialise the struct: fields added later default to 0).
 *  nx, q        cells (8 to 2^30) and quadrature nodes; q must be one of elb_supported_q().
 *  n_herm       order N of the Hermite-expanded equilibrium (Sec. II.D, eq. g_alpha);
 *               0 selects N = q - 1; otherwise 6 <= N <= q - 1 (N >= 6 is what the
 *               Shakhov term needs, Sec. II.D).
 *  length, x0   domain [x0, x0 + length); cell-centred grid x_i = x0 + (i + 1/2) dx.
 *  cfl, dt      dt > 0 is used as given; otherwise dt = cfl * dx / max_k |p_k|.
 *  denseness    E_l = sigma / l at density n_ref and T = 1 (Sec. II.B); 0 is the dilute gas.
 *  kn, kn_length  Knudsen number: Enskog mean free path at n_ref divided by kn_length.
 *  n_ref        reference density of denseness and kn.
 *  pr_mode, pr  ELB_PR_CONST uses pr; ELB_PR_ENSKOG uses the dense-gas Pr(b rho chi)
 *               of Sec. II.B at the local density.
 *  bc           ELB_BC_PERIODIC or ELB_BC_EQUILIBRIUM: three ghost cells per side hold
 *               the equilibrium of ghost_left / ghost_right = (n, u, T) and never change.
 *  closure      0, or 1 to reserve the buffers of the learned closure (q <= 16 only; see
 *               elb_set_closure).  Batches take 0 only.
 *  precision    ELB_FP64: all storage and arithmetic in FP64.
 *               ELB_FP32: FP32 storage and arithmetic, FP64 moment sums.
 *               ELB_FP32_MIXED: as ELB_FP32, plus FP64 per-cell conserved densities
 *               (n, n u, E) advanced by FP64 sums of the fluxes and sources; n, u, T of
 *               every cell are taken from them.
 *  moment_fixup ELB_FP32_MIXED only (ELB_EINVAL otherwise): 1 adds, in every stage, a
 *               fix-up of the FP32 rows that gives them the tracked n, n u, E again
 *               (phi_k += w_k (a + b p_k), theta_k += w_k e, exact on the quadrature) before
 *               they are advected.  This keeps the FP32 distributions from drifting away
 *               from the tracked densities over long runs (heat flux, velocity) at about 5 %
 *               of the step time.  Batches take 0 only.
 *  chi_mode     ELB_CHI_SET: chi = chi_SET(n) of the cell (Sec. II.A, eq. chi).
 *               ELB_CHI_RETFM: revised Enskog theory with the Fischer-Methfessel average
 *               (Sec. II.A, eq. chi_ret): chi = chi_SET(nbar), nbar the density averaged
 *               over a ball of molecular diameter sigma = denseness * kn * kn_length
 *               (E_l = sigma / l); in 1-D nbar(x) = 3/(4 sigma^3) int n(x+s)(sigma^2-s^2) ds
 *               over |s| < sigma, with n between grid points the cubic through the four
 *               nearest points and, beyond the domain, the periodic image or the ghost end
 *               state.  d ln chi is the 6th-order central difference of ln chi.  Needs
 *               sigma / dx <= 128; not with the learned closure (ELB_EUNSUPPORTED
 *               otherwise).  Batches may mix chi_SET and chi_RET-FM instances.  The stage kernel then also reads the
 *               density of J = ceil(sigma / dx) + 1 cells beyond each side of its tile.
 */
typedef struct {
    int32_t nx, q, n_herm;
    double length, x0;
    double cfl, dt;
    double denseness, kn, kn_length, n_ref;
    int32_t pr_mode;
    double pr;
    int32_t bc;
    double ghost_left[3], ghost_right[3];
    int32_t precision;
    int32_t closure;
    int32_t chi_mode;
    int32_t moment_fixup;
} elb_params;

/* Quantities derived from elb_params on the host (for inspection and tests):
 *   out[0] dx, out[1] dt, out[2] b (covolume, eta = b n / 4), out[3] mu_ref (dilute
 *   viscosity at T = 1), out[4] eta at n_ref, out[5] chi_SET at n_ref, out[6] N used.
 * Returns ELB_EINVAL for invalid parameters. */
int elb_derived(const elb_params *p, double out[7]);

/* Number of compiled Q values written to `out` (up to `cap` entries); returns the count. */
int elb_supported_q(int32_t *out, int32_t cap);

/* Gauss-Hermite nodes (roots of He_q, ascending) and weights normalised to sum 1, i.e.
 * for the weight exp(-p^2/2)/sqrt(2 pi) (Sec. II.D).  Host function, pure; q in [1, 256].
 * Nodes come from the eigenvalues of the Jacobi matrix, refined by Newton's method; the
 * weights are the Christoffel numbers 1 / sum_{l<q} He_l(p_k)^2 / l!. */
int elb_quadrature(int32_t q, double *nodes, double *weights);

/* Device workspace needed by a context with these parameters, in bytes (< 0: invalid). */
int64_t elb_workspace_bytes(const elb_params *p);

/* Create a context.  `dev_workspace` is device memory of at least
 * elb_workspace_bytes(p) bytes; `hip_stream` is a hipStream_t or NULL. */
int elb_create(const elb_params *p, void *dev_workspace, int64_t workspace_bytes,
               void *hip_stream, elb_ctx **out);

/* Set the state to the local equilibrium with zero heat flux of the primitive fields
 * n, u, T (host arrays of nx FP64 values; n > 0, T > 0, finite):
 *   phi_k = n g_k(u, T), theta_k = 2 T n g_k(u, T)       (Sec. II.C-D).
 * Returns ELB_EINVAL for invalid values, or when dt exceeds the stability limit of the
 * explicit scheme for this state (CFL > 1 or dt > 2.5 min tau). */
int elb_set_state_moments(elb_ctx *c, const double *n, const double *u, const double *T);

/* Set the state from distributions (host, FP64, nx * q each, row-major [cell][node],
 * quadrature-weighted).  Used for checkpoint restore: in ELB_FP64 a restored run continues
 * bit for bit.  In the FP32 modes the values are rounded to the FP32 storage, and in
 * ELB_FP32_MIXED the tracked conserved densities restart from the sums of the given
 * distributions, so a restart continues the run to FP32 rounding only. */
int elb_set_state_dist(elb_ctx *c, const double *phi, const double *theta);

/* Enqueue nsteps RK3 steps (3 stage launches each) on the context stream.  Asynchronous.
 * With graphs enabled (elb_set_graph), runs of 50 steps or more replay a HIP graph of 50
 * steps captured on the first such call (captured on a private stream, replayed on the
 * context stream); the remainder is launched directly.  Results are bitwise the same as
 * direct launches.  The graph is recaptured after elb_set_state_* and elb_set_closure. */
int elb_step(elb_ctx *c, int64_t nsteps);

/* Step through captured 50-step graphs (enabled = 1) or by direct launches only (0, the
 * default for single contexts: on one MI355X the replay was no faster on small problems
 * and slower on the large shock tube). */
int elb_set_graph(elb_ctx *c, int32_t enabled);

/* Per-cell moments (Sec. II.D) of the current state into host arrays of nx FP64 values;
 * any pointer may be NULL.  Synchronises the stream and reports ELB_ENONFINITE if any
 * stage met an invalid cell since the last check. */
int elb_get_moments(elb_ctx *c, double *n, double *u, double *T, double *qx, double *pxx);

/* Fourier amplitudes of the density of the current state (Sec. IV.A, the projection the
 * sound-wave analysis uses): out[0] = (2/nx) sum_i n_i sin(k x_i) and out[1] = (2/nx)
 * sum_i n_i cos(k x_i), x_i the cell centres.  FP64 sums in a fixed order on the GPU.
 * ELB_EINVAL for NULL out or non-finite k.  Synchronises. */
int elb_get_amplitudes(elb_ctx *c, double k, double out[2]);

/* Copy the distributions to the host (FP64, nx * q each, [cell][node]).  Synchronises. */
int elb_get_dist(elb_ctx *c, double *phi, double *theta);

/* FP64 totals over the interior cells, times dx: mass sum n, momentum sum n u, energy
 * sum (sum_k p_k^2 phi_k + theta_k)/2.  In ELB_FP32_MIXED these are the totals of the
 * tracked FP64 conserved densities.  Synchronises. */
int elb_get_conserved(elb_ctx *c, double out[3]);

/* Time step, number of steps taken since the state was set. */
int elb_get_time(const elb_ctx *c, double *dt, int64_t *steps);

/* Text of the last error on this context (never NULL); with c == NULL, the reason the
 * last failed elb_create, elb_derived, elb_workspace_bytes or elb_mlp_loss_noalloc on the
 * calling thread failed. */
const char *elb_last_error(const elb_ctx *c);

/* Release the context (not the caller's workspace).  Synchronises its stream. */
int elb_destroy(elb_ctx *c);

/* ------------------------------------------------------------------------------------
 * Batches: many independent problems stepped together (one launch per RK3 stage for each
 * group of instances sharing Q, every (instance, tile) item of a group in that launch; a
 * chunk of steps is captured once in a HIP graph and replayed).  Each instance has its own
 * elb_params (nx, q, physics, boundaries, time step); all share `precision`.  Q values
 * with batch kernels: 8, 12, 16, 20, 24, 32, 40, 48, 64, 96, 200.
 * ---------------------------------------------------------------------------------- */
typedef struct elb_batch elb_batch;

/* Device workspace of a batch of `count` instances described by params[0..count-1]. */
int64_t elb_batch_workspace_bytes(const elb_params *params, int32_t count);

/* Create a batch in caller-owned device memory (>= elb_batch_workspace_bytes, 256-byte
 * aligned) on `hip_stream`. */
int elb_batch_create(const elb_params *params, int32_t count, void *dev_workspace,
                     int64_t workspace_bytes, void *hip_stream, elb_batch **out);

/* Equilibrium initial state of instance `inst`, as elb_set_state_moments. */
int elb_batch_set_state_moments(elb_batch *b, int32_t inst, const double *n, const double *u,
                                const double *T);

/* Enqueue nsteps RK3 steps of every instance (each with its own dt).  Asynchronous. */
int elb_batch_step(elb_batch *b, int64_t nsteps);

/* Step through a captured HIP graph (enabled = 1, the default) or by direct launches. */
int elb_batch_set_graph(elb_batch *b, int32_t enabled);

/* Moments / distributions of instance `inst`, as elb_get_moments / elb_get_dist. */
int elb_batch_get_moments(elb_batch *b, int32_t inst, double *n, double *u, double *T,
                          double *qx, double *pxx);
int elb_batch_get_dist(elb_batch *b, int32_t inst, double *phi, double *theta);

/* Tile-shape tuner: for every Q group with more than one compiled tile shape, time the
 * shapes on the current state (stage-1 launches only, which leave the state unchanged) and
 * keep the fastest.  With cache_path != NULL, choices are read from and written to that
 * JSON file (keys "<arch>/<precision>/q<Q>[/ret]/cells2^<k>", "/ret" for chi_RET-FM
 * groups); force = 1 re-times cached keys. */
int elb_batch_tune(elb_batch *b, const char *cache_path, int32_t force);

/* Current groups: Q, strips per block, cells per strip and (instance, tile) items; returns
 * the number of groups (entries beyond `cap` are not written). */
int elb_batch_groups(const elb_batch *b, int32_t *q, int32_t *strips, int32_t *strip_len,
                     int32_t *items, int32_t cap);

/* elb_get_amplitudes of instance `inst`. */
int elb_batch_get_amplitudes(elb_batch *b, int32_t inst, double k, double out[2]);

/* Text of the last error on this batch (never NULL); with b == NULL, the reason the last
 * failed elb_batch_create or elb_batch_workspace_bytes on the calling thread failed. */
const char *elb_batch_last_error(const elb_batch *b);

/* Release the batch (not the caller's workspace).  Synchronises its stream. */
int elb_batch_destroy(elb_batch *b);

/* ------------------------------------------------------------------------------------
 * Learned closure.  A coarse "student" quadrature with Q_s <= 16 nodes carries the Hermite
 * moments 0..Q_s-1 of the distribution (Sec. II.D).  A network predicts, per cell, the part
 * of the right-hand side L[phi] that a fine "teacher" quadrature sees and the student misses:
 *   r = Pi L_T[f_T] - L_s[Pi f_T],  Pi = projection onto the student's nodes that keeps the
 *   Hermite moments 0..Q_s-1 (elb_projection).
 * Inputs (12 per cell): n, u, T, q/(n T^1.5), Pxx/(n T) - 1; the sixth-order central
 * x-derivatives (App. A.3) of n, u, T, q, Pxx times lambda = tau sqrt(T), divided by n,
 * sqrt(T), T, n T^1.5, n T; then E_l and log10(Kn).  Target: y = r tau / n.
 * Network: 12 -> 64 -> 64 -> 64 (SiLU) -> Q_s, bfloat16 weights and layer inputs, FP32
 * accumulation on the matrix cores.  The correction added to L[phi] is
 *   c = P (n / tau) (y out_std + out_mean)
 * with P = I - V (V^T V)^{-1} V^T, V = [1, p, p^2], so that it carries no mass, momentum
 * or energy; cells whose normalised inputs leave [lo, hi] get c = 0 and are counted.
 *
 * Parameters: one packed FP32 array of elb_mlp_param_count() values,
 *   W1 [64][32] (columns 12..31 zero), b1 [64], W2 [64][64], b2 [64], W3 [64][64], b3 [64],
 *   W4 [16][64] (rows >= Q_s zero), b4 [16]   (W[out][in], row-major),
 * and a bfloat16 copy of the same layout (uint16 bit patterns, round to nearest even).
 * Normalisation block: elb_mlp_norm_count() FP32 values,
 *   in_mean[12], in_std[12], out_mean[16], out_std[16], lo[12], hi[12].
 * ---------------------------------------------------------------------------------- */
int64_t elb_mlp_param_count(void);
int64_t elb_mlp_norm_count(void);

/* Device workspace of the training calls for `batch` rows (< 0: invalid batch). */
int64_t elb_mlp_workspace_bytes(int64_t batch);

/* Training calls: device pointers, enqueued on `hip_stream`, asynchronous.
 * forward:  y[b][16] = network((x[index[b]] - in_mean) / in_std) for b < batch (index NULL:
 *           row b); x is [rows][12] FP32.  Keeps the layer inputs in `ws` for backward.
 * loss:     dy = d/dy of mean over b < batch, o < q_out of (y - (t[index[b]] - out_mean) /
 *           out_std)^2 (zero for o >= q_out); *loss (device FP64) = that mean.  t is
 *           [rows][q_out].
 * backward: grad (FP32, packed layout) of sum(dy * y) for the last forward on the same
 *           `ws` and batch; back-propagated signals are rounded to bfloat16 before each
 *           product, biases and SiLU derivatives stay FP32.
 * adam:     one Adam step (Kingma and Ba, 2015) number `step` >= 1 on params, with moment
 *           buffers m, v (zero before step 1); refreshes the bfloat16 copy wb.
 * round:    wb = bfloat16(params). */
int elb_mlp_forward(const float *params, const uint16_t *wb, const float *norm, const float *x,
                    const int32_t *index, int64_t batch, float *y, void *ws, void *hip_stream);
int elb_mlp_loss(const float *y, const float *t, const int32_t *index, const float *norm,
                 int64_t batch, int32_t q_out, float *dy, double *loss, void *ws, void *hip_stream);
int elb_mlp_backward(const uint16_t *wb, const float *dy, int64_t batch, float *grad, void *ws,
                     void *hip_stream);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): elb_mlp_loss without the workspace, with
 * the same arguments, kernels and results.  Its per-block partial sums (at most 256 FP64
 * values) live in a static device array of the library, one copy per GPU, held until the
 * process ends; every call overwrites the entries it reads, so nothing carries over between
 * calls.  The array is shared by all calls on one GPU: calls that overlap on one GPU (other
 * streams, other host threads) race, so serialise them.  The stream must belong to the
 * current device.  No memory is allocated.  ELB_EINVAL for NULL pointers, batch outside
 * [1, 2^24] or q_out outside [1, 16]; ELB_EHIP if the array's address cannot be found;
 * elb_last_error(NULL) gives the reason. */
int elb_mlp_loss_noalloc(const float *y, const float *t, const int32_t *index, const float *norm,
                         int64_t batch, int32_t q_out, float *dy, double *loss, void *hip_stream);

int elb_mlp_adam(float *params, uint16_t *wb, float *m, float *v, const float *grad, int64_t step,
                 float lr, float beta1, float beta2, float eps, void *hip_stream);
int elb_mlp_round(const float *params, uint16_t *wb, void *hip_stream);

/* Host: per-column mean and (population) standard deviation of x [n][dim] (a constant column
 * gets std 1), and with lo, hi != NULL the range of the normalised values widened by
 * margin x (max - min) on each side. */
int elb_mlp_normaliser(const float *x, int64_t n, int32_t dim, double margin, float *mean,
                       float *std_, float *lo, float *hi);

/* Host, pure: the projection Pi [q_to][q_from] (row-major) from q_from to q_to <= q_from
 * Gauss-Hermite nodes: f_s,j = w_j sum_{l<q_to} He_l(p_j) M_l / l! with the teacher's Hermite
 * moments M_l = sum_k He_l(P_k) f_k. */
int elb_projection(int32_t q_from, int32_t q_to, double *P);

/* Host, pure: the lift Lam [q_to][q_from] (row-major) from q_from to q_to >= q_from
 * Gauss-Hermite nodes: f_T,k = W_k sum_{l<q_from} He_l(P_k) M_l / l! with the student's Hermite
 * moments M_l = sum_j He_l(p_j) f_j (Sec. II.D): the Hermite series of the student state on the
 * teacher's nodes.  elb_projection(q_to, q_from) applied after it gives the identity. */
int elb_lift(int32_t q_from, int32_t q_to, double *L);

/* Training along the student's own states: set the teacher's interior distributions to the
 * lift (elb_lift) of the student's current state.  Both FP64, same grid, boundaries and
 * stream; the student was created with closure = 1 and q_student <= q_teacher.  The
 * teacher's ghost rows (its own boundary equilibrium) are kept.  Synchronises. */
int elb_closure_lift(elb_ctx *student, elb_ctx *teacher);

/* Right-hand side L[phi], L[psi] of the current state (host, FP64, nx * q each, [cell][node])
 * of an FP64 context, without the learned correction.  Synchronises; uses the context's
 * stage buffers (the state itself is unchanged). */
int elb_rhs(elb_ctx *c, double *phi_rhs, double *theta_rhs);

/* One training sample per cell from the teacher's current state: the student (FP64,
 * created with closure = 1, same grid and boundaries, same stream, a state already set so
 * that its ghost rows hold its own boundary equilibrium) is set to the projection of the
 * teacher's state, and x [nx][12] (inputs) and y [nx][Q_s] (targets r tau / n) are written
 * to host memory.  Synchronises. */
int elb_closure_sample(elb_ctx *teacher, elb_ctx *student, float *x, float *y);

/* Enable (params and norm on the host, copied) or disable the learned correction of a
 * context created with closure = 1.  When enabled, every stage forms the correction c of
 * its input state and adds a_L dt c to phi.  enabled: 0 off; 1 on, evaluated inside the
 * stage kernel (one launch per stage); 2 on, evaluated by two kernels before each stage
 * (the row moments, then inputs, network and projection) with the same arithmetic, kept
 * as the reference form.  Other values: ELB_EINVAL. */
int elb_set_closure(elb_ctx *c, const float *params, const float *norm, int32_t enabled);

/* Cells (summed over stages) whose inputs left the training range since the counter was
 * last reset; reset = 1 clears it.  Synchronises. */
int elb_closure_outside(elb_ctx *c, int64_t *count, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* ELB_H */
