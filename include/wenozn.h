/* wenozn.h -- C ABI of libwenozn, the MI355X (gfx950) implementation of the hot path of the
 * WENO-ZN finite-difference scheme of Shen, Zhang, Li and Peng, "A novel method for
 * constructing high accurate and robust WENO-Z type scheme" (arXiv 2004.07954).
 *
 * What the library computes
 *   For a conservation law U_t + F(U)_x (+ G(U)_y) = 0 on a uniform grid, the semi-discrete
 *   right-hand side L(U) = -(Fhat_{i+1/2} - Fhat_{i-1/2})/dx [- (Ghat_{j+1/2} - Ghat_{j-1/2})/dy]
 *   (Sec. 2, eq:2; Sec. 4.4, eq:2d), where every interface flux is the fifth-order WENO
 *   reconstruction (eq:3, eq:4) of the Lax-Friedrichs split flux f^{+-} = (F +- alpha U)/2,
 *   component by component, with the Jiang-Shu indicators IS_k (eq:isjiang), the global
 *   indicators tau5 = |IS0 - IS2| (eq:tau) and tau8 (eq:tau8), the adaptive function
 *   C = A ((IS0 + IS2 - tau5 + eps)/(tau5 + eps))^2 (eq:function) and the WENO-ZN weights
 *   alpha_k = c_k (C + tau8/(IS_k + eps)) (eq:new).  f^- is reconstructed from the five points
 *   mirrored about x_{i+1/2} (Sec. 2).  Time integration is the three-stage TVD Runge-Kutta
 *   scheme the paper cites (Sec. 4) with dt = cfl dx / max(|u| + c) from U^n (Sec. 4.3) or
 *   dt = cfl dtx dty / (dtx + dty) in 2D (Sec. 4.4).
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer owned by the caller; the library never
 *     allocates, frees or synchronises (the opt-in p->debug_nonfinite scan excepted).  All
 *     work is enqueued on `stream` (a hipStream_t; NULL = the default stream) and is
 *     asynchronous with respect to the host.
 *   - States are structure-of-arrays fp64: 1D [nvar][n] (nvar = 1 advection, 3 Euler:
 *     rho, rho u, E); 2D [4][ny][nx] with x fastest (rho, rho u, rho v, E).
 *     No ghost cells are stored: the boundary conditions are applied inside the kernels.
 *   - `ws` is a device workspace of at least wzn_workspace_bytes() bytes, 256-byte aligned,
 *     holding the reduction slots of the global Lax-Friedrichs alpha and dt.  Calls that
 *     share one `ws` must be ordered on one stream.
 *   - Arguments are validated before anything is enqueued; on error nothing is enqueued and
 *     a status code is returned (wzn_last_error() then describes it).  No C++ exception
 *     crosses the ABI.  A failed launch returns WZN_ERR_HIP.
 *   - Range: the fp64 weights are evaluated in a single-divide product form whose largest
 *     term grows as the 11th power of the reconstructed values.  Split fluxes F +- alpha U
 *     (wzn_reconstruct: point values) up to 1e26 in magnitude are evaluated correctly; from
 *     about 1e27 (an alternating window) they overflow to non-finite outputs.  The debug mode
 *     (p->debug_nonfinite) reports both the non-finite outputs and states beyond the range
 *     (in fp32 the squared differences of the window reach FLT_MAX from about 1e18, so the
 *     debug mode flags fp32 split fluxes beyond 1e17).
 *     For the same reason eps must lie in [1e-60, 1e50] in fp64 (its fifth power, the
 *     smallest product on a flat stencil, must stay a normal double), and in [1e-36, 1e30]
 *     in fp32; other values return WZN_ERR_ARG.
 */
#ifndef WENOZN_H
#define WENOZN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WZN_ABI_VERSION 2

enum {
  WZN_OK = 0,
  WZN_ERR_ARG = 1,        /* null pointer, bad parameter value */
  WZN_ERR_SIZE = 2,       /* grid too small (n, nx, ny must be >= 6) or too large (1D rows
                             and batched instances <= 2^30 cells, 2D sides <= 2^24) */
  WZN_ERR_DTYPE = 3,      /* unsupported dtype for this entry point */
  WZN_ERR_HIP = 4,        /* a HIP runtime call or kernel launch failed */
  WZN_ERR_NONFINITE = 5,  /* the output holds NaN or Inf (only with p->debug_nonfinite set) */
  WZN_ERR_UNSUPPORTED = 6, /* parameter combination not implemented on the GPU */
  WZN_ERR_NONPHYSICAL = 7, /* an Euler state holds rho <= 0 or p <= 0 (debug_nonfinite only) */
  WZN_ERR_RANGE = 8        /* split fluxes may exceed the range the weights are evaluated for
                              (debug_nonfinite only; see "Range" above) */
};

enum { WZN_ADVECTION = 0, WZN_EULER = 1 };          /* system */
enum { WZN_FP64 = 0, WZN_FP32 = 1 };               /* dtype */
enum { WZN_PERIODIC = 0, WZN_TRANSMISSIVE = 1 };   /* boundary condition per direction */
enum { WZN_SPLIT_LF = 0, WZN_SPLIT_SW = 1 };        /* flux splitting */
enum { WZN_WEIGHTS_ZN = 0, WZN_WEIGHTS_Z = 1 };    /* nonlinear weights */

typedef struct {
  uint32_t abi_version; /* must equal WZN_ABI_VERSION */
  int32_t system;       /* WZN_ADVECTION (1D only) or WZN_EULER */
  int32_t dtype;        /* WZN_FP64 (all entry points) or WZN_FP32 (2D only) */
  int32_t bc_x, bc_y;   /* WZN_PERIODIC or WZN_TRANSMISSIVE; transmissive copies the edge
                           cell into the three ghost cells */
  int32_t p_C;          /* exponent of the ratio inside C (eq:function): must be 2 */
  int32_t q;            /* exponent on tau8/(IS_k+eps) (eq:new): must be 1 */
  int32_t flux_split;   /* WZN_SPLIT_LF (global Lax-Friedrichs, every entry point) or
                           WZN_SPLIT_SW (Steger-Warming, Sec. 4.4: 2D entry points only) */
  double adv_speed;     /* a of u_t + a u_x = 0 (advection only) */
  double gamma;         /* ratio of specific heats, Sec. 4.3: 1.4 */
  double A;             /* constant of eq:function: 10 */
  double eps;           /* epsilon of the weights: 1e-40 (fp64) */
  double lf_alpha_x;    /* < 0: alpha_x = max(|u| + c) of each RHS input (Euler) or |a|
                           (advection); >= 0: this frozen value */
  double lf_alpha_y;    /* same for the y direction (2D) */
  int32_t weights;      /* WZN_WEIGHTS_ZN: the paper's weights (eq:new), every entry point;
                           WZN_WEIGHTS_Z: the WENO-Z weights with q = 1 that the paper compares
                           against (Sec. 2.2, eq:15), alpha_k = c_k (1 + tau5/(IS_k + eps)):
                           wzn_rhs_1d, wzn_rk3_run_1d, wzn_rk3_step_1d and wzn_reconstruct
                           only (others return WZN_ERR_UNSUPPORTED) */
  int32_t debug_nonfinite; /* 0 (default): nothing is checked and nothing synchronises.
                           1: a debugging aid -- after its work every entry point with a
                           workspace synchronises `stream` and checks
                           - the array it writes (dudt, the advanced state, the cotangent):
                             WZN_ERR_NONFINITE if any value is NaN or Inf;
                           - the state it read (right-hand sides, adjoints: u, the stage states
                             or checkpoints; checked before the output, which such a state
                             explains) or wrote (runs; checked after the output):
                             WZN_ERR_NONPHYSICAL if a cell has rho <= 0 or p <= 0 (Euler) or a
                             non-finite value, and, except on the characteristic-field paths,
                             WZN_ERR_RANGE if the bound max|F| + alpha max|U| of its split
                             fluxes (per component and direction; alpha the frozen value or the
                             state's largest wave speed) exceeds 1e26 (fp64) or 1e17 (fp32).
                           wzn_last_error() gives counts and one index.  The work itself has
                           been done when these are returned.  The scans block the host; keep
                           the mode off in production. */
} wzn_params;

/* Fill *p with the paper's values for `system`: A = 10, eps = 1e-40, p_C = 2, q = 1,
 * gamma = 1.4, a = 1, fp64, transmissive (Euler) or periodic (advection), alphas reduced,
 * Lax-Friedrichs split, WENO-ZN weights. */
void wzn_default_params(wzn_params* p, int32_t system);

int32_t wzn_abi_version(void);
const char* wzn_status_string(int32_t status);
/* Message of the last failing call on this host thread ("" if none). */
const char* wzn_last_error(void);

/* Process-wide launch shape of the 1D Euler row kernel: threads per workgroup nt, consecutive
 * cells per thread k, and the layout:
 *   WZN_ROW_LDS_TILE  (0) one tile of nt*k cells per workgroup, both signs of the split flux
 *                     staged in LDS: (256,1), (256,2), (256,4), (128,4), (128,8), (64,1),
 *                     (64,2), (64,4), (64,8);
 *   WZN_ROW_LDS_SPLIT (1) the same tile with the two signs staged one after the other (half
 *                     the LDS): (256,2), (256,4), (128,4), (64,4).
 * (0, 0, any) restores the automatic choice from the grid size.  Set by the autotuner; results
 * do not depend on it (bit for bit).  Returns WZN_ERR_ARG for an unsupported shape. */
enum { WZN_ROW_LDS_TILE = 0, WZN_ROW_LDS_SPLIT = 1 };
int32_t wzn_set_row_tuning(int32_t nt, int32_t k, int32_t layout);

/* The launch shape the 1D entry points use for nvar (1: advection, 3: Euler) components of
 * n cells (the override of wzn_set_row_tuning if set), written to *nt, *k, *layout (host
 * pointers).  WZN_ERR_ARG for a null pointer or another nvar. */
int32_t wzn_get_row_tuning(int32_t nvar, int64_t n, int32_t* nt, int32_t* k, int32_t* layout);

/* Bytes of device workspace `ws` needed by any entry point for grids up to nx * ny cells
 * (ny = 1 in 1D).  Currently a small constant. */
size_t wzn_workspace_bytes(const wzn_params* p, int64_t nx, int64_t ny);

/* ---------------------------------------------------------------- reconstruction
 * wzn_reconstruct: fhat[i] = the fifth-order WENO value at x_{i+1/2} (Sec. 2.1, eq:3 with the
 * candidates of eq:4 and the normalised weights of eq:5) from the five point values
 * f[0 * m + i] .. f[4 * m + i] = f_{i-2} .. f_{i+2}, for 0 <= i < m; the weights are
 * p->weights (WENO-ZN: eq:isjiang, eq:tau, eq:tau8, eq:function, eq:new with p->A, p->eps;
 * or WENO-Z), fp64.  f [5][m] and fhat [m] are device arrays (structure of arrays); the
 * value from the other side of an interface is the same call with the stencil mirrored.
 * m <= 2^34; m = 0 enqueues nothing. */
int32_t wzn_reconstruct(const wzn_params* p, const double* f, double* fhat, int64_t m,
                        void* stream);

/* ---------------------------------------------------------------- 1D
 * wzn_rhs_1d: dudt = L(u) (eq:2) for one state u[nvar][n].  u and dudt must not alias.
 * The LF alpha is p->lf_alpha_x if >= 0, else max over cells of |u| + c (Euler) or |a|. */
int32_t wzn_rhs_1d(const wzn_params* p, const void* u, void* dudt, int64_t n, double dx,
                   void* ws, void* stream);

/* wzn_rhs_1d_noalloc: wzn_rhs_1d without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results (bit for bit) and errors as wzn_rhs_1d; the library's
 * own scratch (the alpha reduction slot and the debug-scan words, 4 KiB whatever n) lives in a
 * static device array, one per GPU, held until the process ends.  Nothing is allocated.  All
 * calls on one GPU share that array: calls that overlap on one GPU (other streams or host
 * threads) race on it and must be serialised by the caller.  Sizes as wzn_rhs_1d (n <= 2^30);
 * WZN_ERR_HIP if the array's device address cannot be taken. */
int32_t wzn_rhs_1d_noalloc(const wzn_params* p, const void* u, void* dudt, int64_t n, double dx,
                           void* stream);

/* One GPU's share of a slab decomposition of a 1D Euler row.
 * wzn_speed_max_1d: *speed1 = max over the cells of u [3][n] of |u| + c (device double): the
 *   per-shard maximum that an all-reduce (MAX) turns into the global Lax-Friedrichs alpha
 *   and the CFL dt (Sec. 4.3).
 * wzn_rhs_1d_slab: dudt = L(u) for a slab of n cells of a longer row, u and dudt [3][n].  The
 *   three cells before it come from ghost_lo and the three after it from ghost_hi ([3][3]
 *   each, component major, in cell order: ghost_lo[c][2] is the cell just before cell 0,
 *   ghost_hi[c][0] the cell just after cell n-1), as a neighbour would send them (or as
 *   p->bc_x would make them at the ends of the whole row).  alpha: device pointer to the
 *   global alpha of the whole row.  Equals the same cells of wzn_rhs_1d on the whole row bit
 *   for bit when the ghost cells and alpha are those of the whole row. */
int32_t wzn_speed_max_1d(const wzn_params* p, const void* u, int64_t n, double* speed1,
                         void* ws, void* stream);
int32_t wzn_rhs_1d_slab(const wzn_params* p, const void* u, const void* ghost_lo,
                        const void* ghost_hi, void* dudt, int64_t n, double dx,
                        const double* alpha, void* ws, void* stream);

/* wzn_rk3_run_1d: advance u[nvar][n] in place by `nsteps` TVD-RK3 steps.
 *   stage   device scratch of 2 * nvar * n elements (the intermediate stage states).
 *   dt_in   NULL: dt = cfl dx / max(|u| + c) of U^n (Sec. 4.3; |a| for advection);
 *           else device array [nsteps] of step sizes.
 *   alpha_in NULL: LF alpha from p->lf_alpha_x (reduced per stage if < 0);
 *           else device array [3 * nsteps] of frozen per-stage alphas.
 *   dt_out, alpha_out  NULL or device arrays [nsteps] / [3 * nsteps] receiving the dt of
 *           every step and the alpha of every stage.
 * The whole run is enqueued as 1 + 3 * nsteps kernels with no host synchronisation, so it
 * can be captured in a HIP graph. */
int32_t wzn_rk3_run_1d(const wzn_params* p, void* u, void* stage, int64_t n, double dx,
                       double cfl, int32_t nsteps, const double* dt_in, const double* alpha_in,
                       double* dt_out, double* alpha_out, void* ws, void* stream);

/* wzn_rk3_step_1d: one step; same as wzn_rk3_run_1d with nsteps = 1. */
int32_t wzn_rk3_step_1d(const wzn_params* p, void* u, void* stage, int64_t n, double dx,
                        double cfl, const double* dt_in, double* dt_out, void* ws,
                        void* stream);

/* ---------------------------------------------------------------- 1D Euler, characteristic fields
 * The paper's 1D Euler setup (Sec. 4.3): the Lax-Friedrichs split and the WENO-ZN
 * reconstruction are carried out in local characteristic fields.  For the interface x_{i+1/2}
 * the flux Jacobian is diagonalised at the Roe average of U_i and U_{i+1}: R has the right
 * eigenvectors (1, u - c, H - u c), (1, u, u^2/2), (1, u + c, H + u c) as columns and
 * Lc = R^{-1}; the cells i-2 .. i+3 are projected with that Lc, field k is split with its own
 * global alpha_k = max over cells of |lambda_k|, lambda = (u - c, u, u + c), reconstructed as
 * in wzn_rhs_1d, and Fhat = R ghat.  Requires p->system == WZN_EULER, fp64.
 *
 * wzn_rhs_1d_char: dudt = L(u) for u[3][n]; u and dudt must not alias.
 *   alpha3  NULL: the three alphas are p->lf_alpha_x (all three) if >= 0, else reduced from u;
 *           else a device array [3] of per-field alphas used as given. */
int32_t wzn_rhs_1d_char(const wzn_params* p, const void* u, void* dudt, int64_t n, double dx,
                        const double* alpha3, void* ws, void* stream);

/* wzn_rk3_run_1d_char: advance u[3][n] in place by `nsteps` TVD-RK3 steps of the
 * characteristic scheme; the arguments are those of wzn_rk3_run_1d except that the alphas
 * come in triples:
 *   alpha_in  NULL (reduced per stage from each stage input, or p->lf_alpha_x for all if >= 0)
 *             or a device array [nsteps][3 stages][3 fields] of frozen alphas;
 *   alpha_out NULL or a device array [nsteps][3][3] receiving them;
 *   dt = cfl dx / max(|u| + c) of U^n unless dt_in is given.
 * Enqueued as 2 + 3 * nsteps kernels with no host synchronisation. */
int32_t wzn_rk3_run_1d_char(const wzn_params* p, void* u, void* stage, int64_t n, double dx,
                            double cfl, int32_t nsteps, const double* dt_in,
                            const double* alpha_in, double* dt_out, double* alpha_out, void* ws,
                            void* stream);

/* ---------------------------------------------------------------- 2D (Euler, Sec. 4.4)
 * Dimension by dimension: L = -(Fhat_{i+1/2,j} - Fhat_{i-1/2,j})/dx - (Ghat_{i,j+1/2} -
 * Ghat_{i,j-1/2})/dy (eq:2d), each a 1D WENO-ZN reconstruction, component by component, of
 * the split flux along its direction:
 *   p->flux_split == WZN_SPLIT_LF: Lax-Friedrichs with its own global alpha
 *     (alpha_x = max(|u| + c), alpha_y = max(|v| + c));
 *   p->flux_split == WZN_SPLIT_SW: Steger-Warming flux-vector splitting, the paper's 2D
 *     setup: F^{+-} = R diag((lambda +- |lambda|)/2) R^{-1} U per cell with the eigenvalues
 *     (u_n - c, u_n, u_n, u_n + c) of the flux Jacobian along the direction (no alphas; the
 *     lf_alpha fields are ignored).
 * p->dtype selects fp64 (arrays of double) or fp32 (arrays of float; the weights use a
 * scale-safe normalisation and eps must be >= 1e-36, e.g. 1e-30).
 * u, dudt: [4][ny][nx], x fastest; bc_x / bc_y select the boundary in each direction.
 *
 * wzn_rhs_2d: dudt = L(u); u and dudt must not alias (dudt is also used as scratch). */
int32_t wzn_rhs_2d(const wzn_params* p, const void* u, void* dudt, int64_t nx, int64_t ny,
                   double dx, double dy, void* ws, void* stream);

/* One GPU's share of a row decomposition of the 2D grid.
 * wzn_speed_max_2d: speed2[0] = max over the cells of u [4][ny][nx] of |u| + c, speed2[1] =
 *   max of |v| + c (device doubles): the per-shard maxima that an all-reduce (MAX) over the
 *   shards turns into the global alphas of the Lax-Friedrichs split (Sec. 4.4) and the CFL dt.
 * wzn_rhs_2d_strip: dudt = L(u) for a strip of ny rows of a larger grid (u, dudt:
 *   [4][ny][nx]).  The y sweep takes the three rows below the strip from ghost_lo and the three
 *   above from ghost_hi ([4][3][nx] each, nearest row last / first: ghost_lo row 2 is the row
 *   just below row 0, ghost_hi row 0 the row just above row ny-1), as a neighbour would send
 *   them (or as p->bc_y would make them at the edge of the whole grid); p->bc_x applies in x.
 *   alpha2: device [2], the global (alpha_x, alpha_y) of the whole grid (required for the
 *   Lax-Friedrichs split, unused by Steger-Warming).  The rows of a strip equal the same rows
 *   of wzn_rhs_2d on the whole grid bit for bit when the ghost rows and alphas are those of
 *   the whole grid.  ny >= 6; u and dudt must not alias (dudt is also scratch). */
int32_t wzn_speed_max_2d(const wzn_params* p, const void* u, int64_t nx, int64_t ny,
                         double* speed2, void* ws, void* stream);
int32_t wzn_rhs_2d_strip(const wzn_params* p, const void* u, const void* ghost_lo,
                         const void* ghost_hi, void* dudt, int64_t nx, int64_t ny, double dx,
                         double dy, const double* alpha2, void* ws, void* stream);

/* wzn_rk3_run_2d: advance u in place by `nsteps` TVD-RK3 steps.
 *   stage  device scratch of 2 * 4 * nx * ny elements of the dtype.
 *   dt_in  NULL: dt = cfl dtx dty / (dtx + dty), dtx = dx / max(|u|+c), dty = dy / max(|v|+c)
 *          of U^n (Sec. 4.4); else device array [nsteps].
 *   dt_out NULL or device array [nsteps] receiving every step's dt.
 * Alphas are reduced per stage unless p->lf_alpha_x / lf_alpha_y are >= 0.
 * Enqueued as 2 + 6 * nsteps kernels with no host synchronisation. */
int32_t wzn_rk3_run_2d(const wzn_params* p, void* u, void* stage, int64_t nx, int64_t ny,
                       double dx, double dy, double cfl, int32_t nsteps, const double* dt_in,
                       double* dt_out, void* ws, void* stream);

/* wzn_rk3_step_2d: one step; same as wzn_rk3_run_2d with nsteps = 1. */
int32_t wzn_rk3_step_2d(const wzn_params* p, void* u, void* stage, int64_t nx, int64_t ny,
                        double dx, double dy, double cfl, const double* dt_in, double* dt_out,
                        void* ws, void* stream);

/* ---------------------------------------------------------------- 2D, characteristic fields
 * The 2D scheme above with each sweep's reconstruction in local characteristic fields: the
 * procedure of Sec. 4.3 (wzn_rhs_1d_char) applied along x and along y.  At each interface the
 * flux Jacobian along the sweep is taken at the Roe average of the two neighbouring states
 * (u, v, H weighted by sqrt(rho)); its eigenvalues are u_n - c, u_n, u_n, u_n + c.  The six
 * stencil cells are projected with its left eigenvectors and split field by field with the
 * Lax-Friedrichs alphas alpha_k = max over the cells of |lambda_k| (x sweep: |u - c|, |u|, |u|,
 * |u + c|; y sweep: the same with v), reconstructed with WENO-ZN and mapped back with the
 * right eigenvectors.  fp64 only, p->flux_split must be WZN_SPLIT_LF and p->weights
 * WZN_WEIGHTS_ZN (else WZN_ERR_DTYPE / WZN_ERR_UNSUPPORTED).
 *
 * work: device scratch of wzn_char2d_work_doubles(nx, ny) doubles (one state: the y part of
 * L), distinct from the other arrays. */
int64_t wzn_char2d_work_doubles(int64_t nx, int64_t ny);

/* wzn_rhs_2d_char: dudt = L(u) for u[4][ny][nx].  alpha8: NULL (reduced from u, or the
 * constants p->lf_alpha_x / p->lf_alpha_y for every field when both are >= 0) or a device
 * array of 8 frozen alphas, the four fields of the x sweep then the four of the y sweep. */
int32_t wzn_rhs_2d_char(const wzn_params* p, const void* u, void* dudt, void* work, int64_t nx,
                        int64_t ny, double dx, double dy, const double* alpha8, void* ws,
                        void* stream);

/* wzn_rk3_run_2d_char: advance u[4][ny][nx] in place by `nsteps` TVD-RK3 steps of the
 * characteristic scheme; stage: device scratch of 2 * 4 * nx * ny doubles; dt as in
 * wzn_rk3_run_2d (dt_in / dt_out as there).  The alphas are reduced from every stage input
 * (p->lf_alpha_x and p->lf_alpha_y must be < 0).  Enqueued as 2 + 6 * nsteps kernels with
 * no host synchronisation. */
int32_t wzn_rk3_run_2d_char(const wzn_params* p, void* u, void* stage, void* work, int64_t nx,
                            int64_t ny, double dx, double dy, double cfl, int32_t nsteps,
                            const double* dt_in, double* dt_out, void* ws, void* stream);

/* ---------------------------------------------------------------- batched 1D Euler
 * Many independent 1D Euler problems of uneven length, advanced by `nsteps` TVD-RK3 steps in
 * ONE persistent kernel launch (plus a one-word counter reset).  Instance i occupies cells
 * offsets[i] .. offsets[i+1]-1 of the concatenated state u[3][total] (component c of cell j
 * at u[c * total + j]); each instance has its own grid spacing dx[i], its own per-stage
 * global Lax-Friedrichs alpha (max |u| + c over the instance) and its own
 * dt = cfl dx[i] / max(|u| + c) of its U^n (Sec. 4.3).  p->bc_x applies to every instance;
 * alphas are always reduced (p->lf_alpha_x must be < 0).
 *   total    cells of all instances together, at most 2^30 (WZN_ERR_SIZE beyond).
 *   stage    device scratch of 2 * 3 * total doubles.
 *   offsets  device int64 [batch + 1], non-decreasing, offsets[batch] == total; every instance
 *            must have 6 .. 2^30 cells (other or out-of-range instances are skipped unchanged).
 *            Decreasing offsets make instances overlap, and two workgroups would then race on
 *            the shared cells; the library does not check this (the Python binding does).
 *   dx       device double [batch].
 *   order    device int32 [batch]: the order in which instances are handed to workgroups
 *            (longest first balances the load), or NULL for 0 .. batch-1.  It must be a
 *            permutation of 0 .. batch-1: an entry outside that range is skipped, and a
 *            repeated entry makes two workgroups advance the same instance at once (a race;
 *            not checked on the device, checked by the Python binding).
 *   tuning   host struct (NULL: defaults); nt in {64, 128, 256} threads per workgroup, k in
 *            {1, 2, 4} cells per thread; layout WZN_ROW_LDS_TILE (pairs 64x2, 64x4, 128x2,
 *            128x4, 256x1, 256x2, 256x4) or WZN_ROW_LDS_SPLIT (128x4, 256x2, 256x4), as for
 *            wzn_set_row_tuning; blocks_per_cu <= 0 takes the occupancy limit.  Results do not
 *            depend on the tuning (bit for bit).
 *   dt_out   NULL or device double [batch][nsteps] receiving every instance's dt history. */
typedef struct {
  int32_t nt;
  int32_t k;
  int32_t blocks_per_cu;
  int32_t layout;
} wzn_batch_tuning;

int32_t wzn_batched_rk3_run_1d(const wzn_params* p, void* u, void* stage, int64_t total,
                               const int64_t* offsets, const double* dx, const int32_t* order,
                               int32_t batch, int32_t nsteps, double cfl,
                               const wzn_batch_tuning* tuning, double* dt_out, void* ws,
                               void* stream);

/* ---------------------------------------------------------------- discrete adjoint (1D Euler)
 * Vector-Jacobian products of the maps the forward entry points evaluate, with the
 * Lax-Friedrichs alpha of every stage and the dt of every step frozen (constants recorded by
 * the forward run).  fp64 only.
 *
 * wzn_rhs_1d_vjp: out = J(u)^T mu, J = dL/dU at u (eq:2 with the WENO-ZN fluxes of Sec. 3).
 *   alpha = p->lf_alpha_x if >= 0, else max(|u| + c) of u, held constant.  All arrays
 *   [3][n]; out must not alias u or mu. */
int32_t wzn_rhs_1d_vjp(const wzn_params* p, const void* u, const void* mu, void* out, int64_t n,
                       double dx, void* ws, void* stream);

/* wzn_rk3_step_1d_vjp: lam_prev = (dU^{n+1}/dU^n)^T lam_next for one TVD-RK3 step.
 *   stages   [3][3][n]: U^n, U1, U2 of the step (as the forward computed them).
 *   scratch  device scratch of 3 * 3 * n doubles.
 *   dt       device pointer to the step's dt; alpha3: device pointer to its 3 stage alphas.
 * Three fused kernels:
 *   lam2 = 2/3 (lam3 + dt J(U2)^T lam3), lam1 = 1/4 (lam2 + dt J(U1)^T lam2),
 *   lam_prev = 1/3 lam3 + 3/4 lam2 + lam1 + dt J(U^n)^T lam1.
 * lam_prev must not alias lam_next, stages or scratch. */
int32_t wzn_rk3_step_1d_vjp(const wzn_params* p, const void* stages, const void* lam_next,
                            void* lam_prev, void* scratch, int64_t n, double dx,
                            const double* dt, const double* alpha3, void* ws, void* stream);

/* wzn_rk3_adjoint_1d_work_doubles: size (in doubles) of `work` for wzn_rk3_adjoint_1d. */
int64_t wzn_rk3_adjoint_1d_work_doubles(int64_t n, int32_t ckpt_every);

/* wzn_rk3_adjoint_1d: the whole reverse pass of an nsteps TVD-RK3 run with checkpointed
 * recomputation, in one call (everything enqueued on `stream`, no host synchronisation).
 *   ckpts    [nseg][3][n], nseg = ceil(nsteps / ckpt_every): state before steps 0,
 *            ckpt_every, 2 ckpt_every, ... (as recorded by the forward run).
 *   dts      device [nsteps]; alphas: device [nsteps][3] (the forward's recorded schedule).
 *   lam      [3][n], in: dJ/dU_T; out: dJ/dU_0.
 *   work     device scratch of wzn_rk3_adjoint_1d_work_doubles(n, ckpt_every) doubles.
 * Per segment, last to first: the stage states of its steps are recomputed from the checkpoint
 * with the frozen schedule, then the step adjoints of wzn_rk3_step_1d_vjp run in reverse. */
int32_t wzn_rk3_adjoint_1d(const wzn_params* p, const void* ckpts, int32_t nsteps,
                           int32_t ckpt_every, const double* dts, const double* alphas,
                           void* lam, void* work, int64_t n, double dx, void* ws, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* WENOZN_H */
