/*
 * crk.h - C ABI of the MI355X CRKSPH neighbour-pair library (libcrk.so).
 *
 * The library evaluates, for one set of gas particles in a periodic cube,
 * the CRKSPH hydro passes of CRK-HACC (arXiv:2511.21921):
 *
 *   smoothing length h   : root of the Thacker neighbour condition
 *                          Delta_N = 1, Delta_N^3 = V n_h^3 / h^3
 *                          (App. A.3, eq. thacker), or h held fixed;
 *   volume V             : V_i^-1 = m_i^-1 sum_j m_j W(|x_ij|, h_i)
 *                          (App. A.2, eq. Vg);
 *   corrections A, B     : the reproducing-kernel coefficients of
 *   and their gradients    W^R_ij = A_i (1 + B_i . x_ij) W_ij(h_i)
 *                          (App. A.1, eq. RK), from the local geometric
 *                          moments, with the 3x3 second-moment solve in FP64;
 *   density rho          : sum m_j V_j W^R_ij / sum V_j^2 W^R_ij
 *                          (Sec. 2.5.1, eq. rhow, gas-only form);
 *   velocity gradient    : -sum_j V_j (v_i - v_j) (x) grad W^R_ij
 *                          (App. A.1, eq. gradv);
 *   accel, du/dt         : pairwise momentum and compatible energy with a
 *                          limited artificial viscosity (Sec. 2.1), optional
 *                          RK relaxation of a pair (App. A.1).
 *
 * and the reverse-mode derivative (adjoint) of a loss
 * L = sum_i g_accel_i . accel_i + sum_i g_dudt_i dudt_i
 * with respect to positions, velocities, internal energies and the
 * viscosity coefficients alpha, beta.
 *
 * Conventions shared by every entry point:
 *  - Arrays are structure-of-arrays in the caller's particle order:
 *    a vector field is [3][n] (component-major), gradB is [9][n] with row
 *    g*3+a = d_g B^a, gradv is [9][n] with row a*3+g = d_g v^a.
 *  - Every array argument is a DEVICE pointer owned by the caller; the
 *    library never frees or retains caller memory beyond the call.
 *  - "Real" arrays are float in CRK_FP32 mode and double in CRK_FP64 mode;
 *    positions, accelerations, du/dt and all gradients are always double.
 *  - Work is enqueued on the given HIP stream (hipStream_t passed as void*,
 *    NULL = default stream). The call may synchronise that stream to read
 *    small control values (the largest h, overflow and capping flags).
 *  - A crk_ctx is not thread-safe; use one context per stream.
 *  - Status codes: CRK_OK on success; CRK_EINVAL for a null pointer,
 *    negative n or a bad parameter; CRK_EDOMAIN when a smoothing length
 *    reaches half the box (minimum image undefined); CRK_ENOMEM when device
 *    memory cannot be allocated; CRK_EHIP for any other HIP runtime error;
 *    CRK_ENOTCONV when the h solve did not converge for some particle (the
 *    outputs are still written); CRK_ENONFINITE when check_finite is set and
 *    an output is not finite. crk_last_error() gives a readable message.
 */
#ifndef CRK_H
#define CRK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct crk_ctx crk_ctx;

typedef enum {
  CRK_OK = 0,
  CRK_EINVAL = -1,
  CRK_ENOMEM = -2,
  CRK_EHIP = -3,
  CRK_EDOMAIN = -4,
  CRK_ENOTCONV = -5,
  CRK_ENONFINITE = -6
} crk_status;

typedef enum { CRK_CUBIC_SPLINE = 0, CRK_WENDLAND_C4 = 1 } crk_kernel;

/* CRK_FP32: FP32 pair arithmetic, FP64 correction solve and force/energy
 * accumulators (the paper's single-precision force kernels, App. A.4).
 * CRK_FP64: every step in FP64. */
typedef enum { CRK_FP32 = 0, CRK_FP64 = 1 } crk_precision;

typedef struct {
  double box;        /* periodic cube side L > 0 */
  double gamma;      /* adiabatic index, 5/3 (Sec. 2.4.1) */
  double alpha;      /* viscosity linear coefficient */
  double beta;       /* viscosity quadratic coefficient */
  double eps2;       /* viscosity softening, e.g. 0.01 */
  double n_h;        /* particles per kernel radius; N = 4 pi/3 n_h^3 (App. A.2) */
  int kernel;        /* crk_kernel; support radius h (App. A.2) */
  int precision;     /* crk_precision */
  int h_mode;        /* 0: h is an input; 1: solve for h (input = first guess) */
  int h_max_iter;    /* Newton/bisection iteration cap, e.g. 60 */
  double h_rtol;     /* relative h tolerance, e.g. 1e-6 (FP32), 1e-13 (FP64) */
  double dt_relax;   /* RK relaxation time step (App. A.1); 0 disables */
  int store_corrections; /* 1: keep moments for the adjoint; 0: recompute them */
  int check_finite;  /* 1: count non-finite outputs and fail with CRK_ENONFINITE */
  int timing;        /* 1: time every pass with HIP events (see crk_pass_times) */
  int search;        /* neighbour search: 0 automatic, 1 periodic cell list (cells of at least
                        0.625 x the largest h, a 5x5x5 stencil), 2 tree of Morton-ordered
                        16-particle leaves (for smoothing lengths spanning orders of
                        magnitude); automatic uses the cell list unless a cell holds more
                        than max(1024, 16 x the mean occupancy) particles or a particle more
                        than max(1024, 16 x the expected count) candidates */
} crk_params;

typedef struct {
  long long n_pairs_gather; /* sum_i |{j != i : r_ij < h_i}| */
  long long n_pairs_force;  /* sum_i |{j != i : r_ij < max(h_i, h_j)}| */
  int h_iter_max;           /* largest Newton/bisection count */
  int h_unconverged;        /* particles whose h solve hit the iteration cap */
  int m2_singular;          /* particles with a singular second moment (uncorrected kernel) */
  int relaxed;              /* particles flagged by the relaxation criterion */
  int nonfinite;            /* non-finite outputs (check_finite only) */
  int grid;                 /* cells per box side used by the cell list */
  int speculative;          /* 1: this forward ran on the previous one's cell-list geometry
                               and was accepted by its single end-of-call check */
  long long n_candidates;   /* candidate pairs the neighbour search kept: the cell list's
                               pairs within the cut of the solved h; the tree's pairs
                               within each search radius (padded beyond the FP32 rounding
                               of the leaf tests), summed over its retry rounds */
  long long n_searched;     /* particles the neighbour search launches took (n per cell-list
                               search; the particles of every tree round) */
} crk_stats;

/* Fills *p with the defaults for the given precision. */
void crk_default_params(crk_params *p, int precision);

/* Creates a context; *ctx receives it. Validates p (box > 0, n_h > 0,
 * kernel and precision in range). Allocates nothing on the device. */
crk_status crk_create(crk_ctx **ctx, const crk_params *p);

/* Replaces the parameters of an existing context. A change of any field
 * other than timing and check_finite drops the state kept for crk_backward
 * (a following crk_backward returns CRK_EINVAL until the next forward), so
 * an adjoint is always taken with the parameters of its forward. */
crk_status crk_set_params(crk_ctx *ctx, const crk_params *p);

/* Pre-allocates device workspace for up to n_max particles so that later
 * calls with n <= n_max allocate only if a neighbour list outgrows it. When
 * this grows a buffer the forward state kept for crk_backward is dropped. */
crk_status crk_reserve(crk_ctx *ctx, long long n_max);

/* Releases the context and all workspace it owns. NULL is accepted. */
crk_status crk_destroy(crk_ctx *ctx);

/* Readable message of the last failing call on ctx ("" if none). */
const char *crk_last_error(const crk_ctx *ctx);

/* Forward evaluation.
 *   x      [3][n] double  positions; wrapped into [0, box) internally
 *   v      [3][n] Real    velocities
 *   m      [n] Real       masses (> 0)
 *   u      [n] Real       specific internal energies (> 0)
 *   h      [n] Real       in: fixed h (h_mode 0) or first guess (h_mode 1);
 *                         out: the h used (solved in h_mode 1)
 *   V, rho [n] Real       volume and density
 *   A      [n] Real, B [3][n], gradA [3][n], gradB [9][n]  corrections
 *   gradv  [9][n] Real    velocity gradient
 *   accel  [3][n] double  dv/dt from the hydro pairs
 *   dudt   [n] double     du/dt (compatible energy)
 *   stats  host pointer or NULL; when given, the call synchronises the
 *          stream and fills it.
 * Host reads: a forward reads device counters to size the cell list and its
 * lists (input check, clustering test, h solve, list capacities). After a
 * forward that settled on the cell list at its first grid, the next one with
 * the same n and precision launches every pass with that geometry and reads
 * the counters once at the end; when they show that the careful order would
 * have chosen differently (another grid, clustering, an overflow, a capped h
 * root), it runs again the careful way. Either way the outputs are the same.
 * Such a forward keeps the last cell list, without sorting again, once a
 * check has found that no particle had left its cell; a particle that has
 * left it since makes that forward run again the careful way.
 * n = 0 is a no-op returning CRK_OK. Input and output arrays must not
 * overlap. The context keeps the cell list, neighbour list and the sorted
 * intermediates for a following crk_backward. After a status other than
 * CRK_OK, CRK_ENOTCONV and CRK_ENONFINITE the output arrays (h included)
 * are undefined: a speculative attempt may have written them before the
 * failing check. Non-finite positions are rejected with CRK_EINVAL. */
crk_status crk_forward(crk_ctx *ctx, void *hip_stream, long long n, const double *x,
                       const void *v, const void *m, const void *u, void *h, void *V,
                       void *rho, void *A, void *B, void *gradA, void *gradB, void *gradv,
                       double *accel, double *dudt, crk_stats *stats);

/* Reverse-mode derivative of L = sum g_accel . accel + sum g_dudt dudt for
 * the most recent crk_forward on ctx, which must have had the same n (the
 * inputs themselves are taken from the state kept by that forward).
 *   g_accel [3][n] double, g_dudt [n] double   loss weights (device)
 *   g_x [3][n], g_v [3][n], g_u [n]            outputs (device, double)
 *   g_alpha_beta [2]                            output (device, double)
 * With h_mode 1 the smoothing lengths are functions of the positions (the
 * implicit-function term is included); with h_mode 0 they are constants.
 * Masses are constants. Returns CRK_EINVAL if no matching forward exists.
 * The adjoint workspace (428 bytes per FP32 particle, 656 per FP64 one) is
 * carved from the forward's candidate scratch, which is dead once the lists
 * are built, and grows it when smaller. */
crk_status crk_backward(crk_ctx *ctx, void *hip_stream, long long n, const double *g_accel,
                        const double *g_dudt, double *g_x, double *g_v, double *g_u,
                        double *g_alpha_beta);

/* crk_backward with no device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight training or serving loops, harnesses
 * that forbid hipMalloc. Same arguments, results and errors as crk_backward
 * (it runs the same kernels), plus CRK_EINVAL for n above 65,536 particles.
 * The workspace (the adjoint accumulators, packed records and per-block
 * partial sums: 41 MiB, sized for 65,536 FP64 particles) is one static
 * device array of the library, one copy per GPU, held until the process
 * ends; its address on each device is taken on the first call there. Every
 * call on a GPU reuses that array, so calls that overlap on one GPU (other
 * streams, contexts or threads) race: the caller serialises them. Nothing
 * in it needs to start at zero (every element is written before it is
 * read). Pass times are not recorded. For a whole step without allocation,
 * size the context with crk_reserve before the forward. */
crk_status crk_backward_noalloc(crk_ctx *ctx, void *hip_stream, long long n,
                                const double *g_accel, const double *g_dudt, double *g_x,
                                double *g_v, double *g_u, double *g_alpha_beta);

/* One kick-drift-kick step of length dt on a single timestep level (App. A.4
 * KDK update), with the smoothing length integrated by the combined Thacker
 * and continuity rate and its exponential update (App. A.3):
 *   v^1/2 = v + a dt/2, u^1/2 = u + (du/dt) dt/2;
 *   x <- x + v^1/2 dt in double, wrapped into [0, box);
 *   Delta_N = n_h V^(1/3) / h, h^T = h (1 - lambda + lambda Delta_N),
 *   hdot = (h^T - h)/dt + h div(v)/3, h <- h exp(hdot dt / h);
 *   the forward at (x, v^1/2 + a dt/2, m, u^1/2 + (du/dt) dt/2, h), h fixed;
 *   v = v^1/2 + a^1 dt/2, u = u^1/2 + (du/dt)^1 dt/2.
 * The context must have h_mode 0 (h is integrated here, not solved).
 *   dt             > 0, finite
 *   thacker_lambda the Thacker weight lambda in [0, 1]
 *   x [3][n] double, v [3][n] Real, u [n] Real, h [n] Real   in/out: the state,
 *                  advanced by dt
 *   m [n] Real     in
 *   V [n], gradv [9][n] Real, accel [3][n], dudt [n] double  in: the forward at
 *                  the current state (a crk_forward or crk_kdk_step on these
 *                  arrays); out: the forward at the new state
 *   rho, A, B, gradA, gradB   out, as in crk_forward
 * All arrays are device memory, caller-owned, in the caller's order; the
 * context's workspace holds the predicted velocity and energy. The forward
 * state is kept for crk_backward, which then differentiates the end-of-step
 * evaluation. Errors: CRK_EINVAL for h_mode != 0, a bad dt or lambda, null
 * arrays or n above 2^25 - 1; otherwise those of crk_forward (after an error
 * the arrays may hold a partly advanced state). n = 0 is a no-op. */
crk_status crk_kdk_step(crk_ctx *ctx, void *hip_stream, long long n, double dt,
                        double thacker_lambda, double *x, void *v, const void *m, void *u,
                        void *h, void *V, void *rho, void *A, void *B, void *gradA, void *gradB,
                        void *gradv, double *accel, double *dudt, crk_stats *stats);

/* One big step dt of the hierarchical kick-drift-kick integrator on
 * power-of-two timestep levels (App. A.4; h, V and rho as in App. A.3).
 * Particle i of level L_i (levels [n] int, device, 0 <= L_i <= 30) is active
 * on intervals dt_a = dt / 2^L_i; all particles drift on dt_min =
 * dt / 2^Lmax, Lmax the largest level. Per particle and interval:
 *   open:  v^1/2 = v + a^0 dt_a/2, u^1/2 = u + (du/dt)^0 dt_a/2,
 *          hdot = (h^T - h)/dt_a + h div(v)/3 from its latest evaluation;
 *   every substep, every particle: x <- x + v_j dt_min in double on the
 *          parabola v_j = v^1/2 + a^0 (t_elapsed + (dt_min - dt_a)/2),
 *          h <- h exp(hdot dt_min / h), V <- (h/n_h)^3,
 *          rho <- rho exp(-div(v) dt_min);
 *   at each substep end, one forward at the predicted velocities and
 *          energies v^1/2 + a^0 t, u^1/2 + (du/dt)^0 t (t from the centre of
 *          the interval) in which the particles whose interval does not end
 *          are passive: they skip the volume, moment, density and force sums
 *          and keep V, rho, grad v and A, B, grad A, grad B from these arrays;
 *   close (interval end): v = v^1/2 + a^1 dt_a/2, u = u^1/2 + (du/dt)^1 dt_a/2,
 *          and the particle's evaluation (accel, dudt, V, rho, A, B, gradA,
 *          gradB, gradv) is stored in the arrays.
 * Timestep refinement (App. A.5; refine_at null: none): refine_at [n] and
 * refine_level [n] (int, device) move particle i with refine_at[i] >= 0 to
 * the finer level refine_level[i] at the start of substep j_r = refine_at[i]
 * (time j_r dt_min; Lmax counts the refinement levels). Its interval opened
 * e before; v and u advance under the constant a^0, du^0 to that time
 * (v <- v + a^0 e) and an interval of the new level opens there as above,
 * so the cycle ends with v^1 = v^0 + a^0 e + (a^0 + a^1) dt_c / 2 (the
 * corrected half kick for e = 0, the piecewise-constant final kick
 * otherwise); the particle keeps the new level to the end of the big step.
 * j_r must lie in [0, 2^Lmax) on the new level's grid (a multiple of
 * 2^(Lmax - refine_level[i])), refine_level[i] in (levels[i], 30].
 * Otherwise levels stay fixed during the call; every interval ends at dt, so
 * the state returned is synchronised. Arrays as in crk_kdk_step, all in/out: on entry
 * the evaluation at the current state (every particle), on return each
 * particle's latest evaluation (all at the new state). With every level 0
 * and no refinement this is crk_kdk_step up to rounding. The context needs h_mode 0; its
 * workspace holds the half-kicked state and hdot. After a call with Lmax > 0
 * crk_backward is not available (the last evaluation had passive
 * particles). Errors: CRK_EINVAL for h_mode != 0, a bad dt or lambda, levels
 * outside [0, 30], a refinement that breaks the rules above, null arrays
 * (refine_level null with refine_at given) or n above 2^25 - 1; otherwise those of
 * crk_forward, from any substep (after such an error the arrays may hold a
 * partly advanced state). The call reads the device once for the level
 * range and the particles per level, once for the refinements, then once per
 * substep (the forward's check at its end, when the substep's forward keeps
 * the cell list and geometry of the one before; more when it must run the
 * careful way). A substep whose end finds few particles active (at most
 * 32,768, counted from the levels) gives each of them a 16-lane row in every
 * pass. n = 0 is a no-op. */
crk_status crk_hkdk_step(crk_ctx *ctx, void *hip_stream, long long n, double dt,
                         double thacker_lambda, const int *levels, const int *refine_at,
                         const int *refine_level, double *x, void *v, const void *m, void *u,
                         void *h, void *V, void *rho, void *A, void *B, void *gradA, void *gradB,
                         void *gradv, double *accel, double *dudt, crk_stats *stats);

/* Tabulated source function of the exact-integration cooling (Sec. 2.2,
 * exact integration): lam[k] at u_k = 10^(log10_u0 + k dex), k = 0 .. K-1,
 * interpolated by piecewise power laws between nodes of the same sign. The
 * composition is folded into the table: Lambda(u; rho) = rho^2 lam(u), so
 * that du/dt = -Lambda / rho = -rho lam(u); lam > 0 cools, lam < 0 heats, and
 * a bin whose end values differ in sign holds an equilibrium. lam is a host
 * array, copied (the call synchronises the stream). The context keeps one
 * table; a new call replaces it. Errors: CRK_EINVAL for K < 2, dex <= 0,
 * non-finite values or energies beyond 10^(+-300). */
crk_status crk_cooling_table(crk_ctx *ctx, void *hip_stream, int K, double log10_u0, double dex,
                             const double *lam);

/* Integrates du/dt = -rho lam(u) exactly over dt for n particles (the table
 * of crk_cooling_table), each with its own anchor u_a = u^0 and fixed rho:
 *   rho [n] Real  in (device), u [n] Real  in/out (device), caller's order.
 * Energies outside the table are clamped to its ends. In a sign-change bin
 * the source is held at the larger edge magnitude and u stops at the zero of
 * the linear interpolant when it moves toward it; moving away from an
 * unstable zero it leaves the bin and continues. Arithmetic is FP64 in both
 * precisions. Errors: CRK_EINVAL without a table, for dt < 0 or not finite,
 * null arrays; n = 0 is a no-op. */
crk_status crk_cool(crk_ctx *ctx, void *hip_stream, long long n, double dt, const void *rho,
                    void *u);

/* Subgrid deposition (App. A.2 eq. (Vsg); Secs. 2.5-2.7 eqs. (windmetal),
 * (Anorm), (starmetal), (stellarmom), (AGNE)): n_src point sources hand mass
 * dM, metal mass dMZ and energy dE to the gas around them, in one call.
 *   Source volume: V_s = (1 - C w(0) / n_h_src^3) / sum_j W(|x_sj|, h_j), the
 *     SPH sum over gas j with |x_sj| < h_j plus the source's own term at
 *     h_s = n_h_src V_s^(1/3) (the fixed point in closed form).
 *   Normalisation: A_s = 1 / sum over eligible gas j with |x_sj| < h_s of
 *     V_j W(|x_sj|, h_s); gas is eligible when mZ_j <= z_max m_j and
 *     m_j <= m_max (pass +inf for no limit). A source with no eligible gas in
 *     reach gets A_s = 0 and deposits nothing; one with no gas at all in reach
 *     also gets V_s = h_s = 0.
 *   Deposition: gas j gains f_sj = A_s V_j W(|x_sj|, h_s) of dM, dMZ and dE of
 *     every source s; the mass arrives with the source velocity v_s
 *     (momentum conserved: v_j <- (m_j v_j + sum f dM v_s) / m_j'), the energy
 *     becomes specific energy of the grown particle (u_j <- (m_j u_j +
 *     sum f dE) / m_j'). Totals are conserved to rounding.
 * Arrays are device memory in the caller's order; Real is float or double by
 * the context precision; positions are double, periodic in the box:
 *   x_gas [3][n_gas], h_gas, V_gas [n_gas] in (V from crk_forward);
 *   m_gas, mZ_gas, u_gas [n_gas], v_gas [3][n_gas] in/out;
 *   x_src [3][n_src], dM, dMZ, dE [n_src], v_src [3][n_src] in;
 *   V_src, h_src, A_src [n_src] out.
 * Sources search one grid of the gas (cells at least the largest gas h) with
 * a stencil as wide as their own radius; their receivers are listed, sorted
 * by gas index (stable) and summed per gas particle in source order: no
 * float atomics, reproducible results. Arithmetic is FP64 in both
 * precisions; the kernel shape is the context's. The call reads counters
 * back to the host twice (synchronises the stream); workspace grows with
 * the number of source-gas pairs (CRK_ENOMEM beyond 2^31).
 * Errors: CRK_EINVAL for negative counts, null arrays, n_h_src^3 <= C w(0),
 * NaN limits, gas h not finite or <= 0; CRK_EDOMAIN when a gas or source
 * smoothing length reaches half the box. n_src = 0 is a no-op. */
crk_status crk_deposit(crk_ctx *ctx, void *hip_stream, long long n_gas, const double *x_gas,
                       const void *h_gas, const void *V_gas, void *m_gas, void *v_gas,
                       void *mZ_gas, void *u_gas, long long n_src, const double *x_src,
                       const void *dM, const void *dMZ, const void *dE, const void *v_src,
                       double n_h_src, double z_max, double m_max, void *V_src, void *h_src,
                       void *A_src);

/* Per-pass device time. Passes are numbered 0 .. crk_pass_count()-1 and
 * named by crk_pass_name(k) (NULL when k is out of range). With
 * params.timing = 1 every pass of crk_forward / crk_backward is bracketed by
 * HIP events recorded on the call's stream; crk_pass_times() waits for the
 * recorded events, writes the accumulated milliseconds of each pass to
 * ms[k] and the number of timed launches to calls[k] (host arrays of
 * crk_pass_count() entries, either may be NULL), and clears the totals when
 * reset != 0. */
int crk_pass_count(void);
const char *crk_pass_name(int k);
crk_status crk_pass_times(crk_ctx *ctx, double *ms, long long *calls, int reset);

#ifdef __cplusplus
}
#endif

#endif /* CRK_H */
