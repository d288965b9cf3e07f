// extern "C" entry points of libwenozn: argument validation, error reporting and dispatch to
// the kernels.  Declarations and the meaning of every argument are in include/wenozn.h.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "wzn_host.hpp"

namespace wzn {

static thread_local char g_err[512] = "";

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(WZN_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return WZN_OK;
}

__global__ void fill_double_kernel(double* p, double v) {
  if (threadIdx.x == 0) p[0] = v;
}

int launch_fill_double(double* p, double v, hipStream_t s) {
  hipLaunchKernelGGL(fill_double_kernel, dim3(1), dim3(64), 0, s, p, v);
  return check_launch("fill_double_kernel");
}

static Tuning1D g_row_override = {0, 0, 0};

Tuning1D row_override() { return g_row_override; }

// Launch shape of the 1D row kernel: the caller's override if set; otherwise, as measured on
// MI355X, 1024-cell tiles with the signs staged one at a time from 3 * 2^18 cells (one round
// of four workgroups per CU at 2^20 cells), 512-cell tiles staged one sign at a time from 2^17
// (5 % faster than both signs at once at 2^18, equal at 2^16), 512-cell tiles with both signs
// from 2^15, else 256-cell tiles.
Tuning1D tuning_1d(int nv, int64_t n) {
  if (nv == 1) return Tuning1D{64, 4, ROW_LDS_TILE};
  if (g_row_override.nt > 0) return g_row_override;
  if (n >= (int64_t)3 << 18) return Tuning1D{256, 4, ROW_LDS_SPLIT};
  if (n >= (int64_t)1 << 17) return Tuning1D{256, 2, ROW_LDS_SPLIT};
  if (n >= (int64_t)1 << 15) return Tuning1D{256, 2, ROW_LDS_TILE};
  return Tuning1D{256, 1, ROW_LDS_TILE};
}

static int check_params(const wzn_params* p, bool allow_fp32, bool allow_z = false) {
  if (!p) return set_error(WZN_ERR_ARG, "params is NULL");
  if (p->abi_version != WZN_ABI_VERSION)
    return set_error(WZN_ERR_ARG, "abi_version %u != %d", p->abi_version, WZN_ABI_VERSION);
  if (p->system != WZN_ADVECTION && p->system != WZN_EULER)
    return set_error(WZN_ERR_ARG, "unknown system %d", p->system);
  if (p->dtype != WZN_FP64 && !(allow_fp32 && p->dtype == WZN_FP32))
    return set_error(WZN_ERR_DTYPE, "dtype %d not supported here", p->dtype);
  if (p->bc_x != WZN_PERIODIC && p->bc_x != WZN_TRANSMISSIVE)
    return set_error(WZN_ERR_ARG, "unknown bc_x %d", p->bc_x);
  if (p->bc_y != WZN_PERIODIC && p->bc_y != WZN_TRANSMISSIVE)
    return set_error(WZN_ERR_ARG, "unknown bc_y %d", p->bc_y);
  if (p->p_C != 2 || p->q != 1)
    return set_error(WZN_ERR_UNSUPPORTED, "only p_C = 2, q = 1 (the paper's weights) run here");
  if (p->flux_split != WZN_SPLIT_LF && p->flux_split != WZN_SPLIT_SW)
    return set_error(WZN_ERR_ARG, "unknown flux_split %d", p->flux_split);
  if (p->weights != WZN_WEIGHTS_ZN && p->weights != WZN_WEIGHTS_Z)
    return set_error(WZN_ERR_ARG, "unknown weights %d", p->weights);
  if (p->debug_nonfinite != 0 && p->debug_nonfinite != 1)
    return set_error(WZN_ERR_ARG, "debug_nonfinite must be 0 or 1");
  if (p->weights == WZN_WEIGHTS_Z && !allow_z)
    return set_error(WZN_ERR_UNSUPPORTED,
                     "the WENO-Z weights run in wzn_rhs_1d, wzn_rk3_run_1d and wzn_reconstruct");
  if (!(p->eps > 0.0) || !(p->A > 0.0))
    return set_error(WZN_ERR_ARG, "eps and A must be positive");
  // the fp64 product form multiplies five eps-sized factors on a flat stencil (the smallest
  // product, which must stay a normal double) and the fp32 form needs 16 eps normal
  if (p->dtype == WZN_FP64 && !(p->eps >= 1e-60 && p->eps <= 1e50))
    return set_error(WZN_ERR_ARG, "fp64 needs 1e-60 <= eps <= 1e50 (got %g)", p->eps);
  if (p->dtype == WZN_FP32 && !(p->eps >= 1e-36 && p->eps <= 1e30))
    return set_error(WZN_ERR_ARG, "fp32 needs 1e-36 <= eps <= 1e30 (got %g)", p->eps);
  if (p->system == WZN_EULER && !(p->gamma > 1.0))
    return set_error(WZN_ERR_ARG, "gamma must exceed 1");
  if (p->system == WZN_ADVECTION && !(p->adv_speed != 0.0) && p->lf_alpha_x < 0.0)
    return set_error(WZN_ERR_ARG, "advection speed must be nonzero");
  return WZN_OK;
}

// The debug_nonfinite mode: after an entry point's work, scan the array it wrote.
static int scanned(int st, const wzn_params* p, const void* x, int64_t count, bool f32,
                   Workspace* w, void* stream) {
  if (st || !p->debug_nonfinite) return st;
  return debug_nonfinite_scan(x, count, f32, w, (hipStream_t)stream);
}

// The debug mode's check of a state after an entry point's work: the state it read (right-hand
// sides, adjoints) or wrote (runs) has rho, p > 0 and split fluxes inside the weights' range
// (the range is not checked for the characteristic-field paths, whose reconstructed values are
// projections of the split fluxes).
static int state_checked(int st, const wzn_params* p, const void* state, int64_t N, int nv,
                         bool f32, bool range, Workspace* w, void* stream) {
  if (st || !p->debug_nonfinite) return st;
  return debug_state_scan(p, state, N, nv, f32, range, w, (hipStream_t)stream);
}

static int check_1d(const wzn_params* p, int64_t n, double dx, void* ws, bool allow_z = false) {
  int st = check_params(p, false, allow_z);
  if (st) return st;
  if (p->flux_split != WZN_SPLIT_LF)
    return set_error(WZN_ERR_UNSUPPORTED, "the 1D entry points use the Lax-Friedrichs split");
  if (n < 6) return set_error(WZN_ERR_SIZE, "n = %lld < 6", (long long)n);
  if (n > (int64_t)1 << 30)
    return set_error(WZN_ERR_SIZE, "n = %lld > 2^30 cells per row", (long long)n);
  if (!(dx > 0.0)) return set_error(WZN_ERR_ARG, "dx must be positive");
  if (!ws) return set_error(WZN_ERR_ARG, "workspace is NULL");
  if (((uintptr_t)ws) & 255) return set_error(WZN_ERR_ARG, "workspace not 256-byte aligned");
  return WZN_OK;
}

static int check_2d(const wzn_params* p, int64_t nx, int64_t ny, double dx, double dy, void* ws) {
  int st = check_params(p, true);
  if (st) return st;
  if (p->system != WZN_EULER) return set_error(WZN_ERR_ARG, "2D supports the Euler system only");
  if (nx < 6 || ny < 6)
    return set_error(WZN_ERR_SIZE, "nx = %lld, ny = %lld: both must be >= 6", (long long)nx,
                     (long long)ny);
  if (nx > (1 << 24) || ny > (1 << 24) || nx * ny > ((int64_t)1 << 36))
    return set_error(WZN_ERR_SIZE, "grid %lld x %lld too large", (long long)nx, (long long)ny);
  if (!(dx > 0.0) || !(dy > 0.0)) return set_error(WZN_ERR_ARG, "dx and dy must be positive");
  if (!ws) return set_error(WZN_ERR_ARG, "workspace is NULL");
  if (((uintptr_t)ws) & 255) return set_error(WZN_ERR_ARG, "workspace not 256-byte aligned");
  return WZN_OK;
}

}  // namespace wzn

using namespace wzn;

extern "C" {

void wzn_default_params(wzn_params* p, int32_t system) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->abi_version = WZN_ABI_VERSION;
  p->system = system;
  p->dtype = WZN_FP64;
  p->bc_x = p->bc_y = system == WZN_ADVECTION ? WZN_PERIODIC : WZN_TRANSMISSIVE;
  p->p_C = 2;
  p->q = 1;
  p->adv_speed = 1.0;
  p->gamma = 1.4;
  p->A = 10.0;
  p->eps = 1e-40;
  p->lf_alpha_x = -1.0;
  p->lf_alpha_y = -1.0;
}

int32_t wzn_abi_version(void) { return WZN_ABI_VERSION; }

const char* wzn_status_string(int32_t status) {
  switch (status) {
    case WZN_OK: return "ok";
    case WZN_ERR_ARG: return "invalid argument";
    case WZN_ERR_SIZE: return "invalid size";
    case WZN_ERR_DTYPE: return "unsupported dtype";
    case WZN_ERR_HIP: return "HIP error";
    case WZN_ERR_NONFINITE: return "non-finite output";
    case WZN_ERR_UNSUPPORTED: return "unsupported parameters";
    case WZN_ERR_NONPHYSICAL: return "non-physical state";
    case WZN_ERR_RANGE: return "values beyond the evaluated range";
    default: return "unknown status";
  }
}

const char* wzn_last_error(void) { return g_err; }

int32_t wzn_set_row_tuning(int32_t nt, int32_t k, int32_t layout) {
  g_err[0] = 0;
  if (nt == 0 && k == 0) {
    g_row_override = Tuning1D{0, 0, 0};
    return WZN_OK;
  }
  bool ok;
  if (layout == ROW_LDS_TILE)
    ok = (nt == 256 && (k == 1 || k == 2 || k == 4)) || (nt == 128 && (k == 4 || k == 8)) ||
         (nt == 64 && (k == 1 || k == 2 || k == 4 || k == 8));
  else if (layout == ROW_LDS_SPLIT)
    ok = (nt == 256 && (k == 2 || k == 4)) || ((nt == 128 || nt == 64) && k == 4);
  else
    ok = false;
  if (!ok)
    return set_error(WZN_ERR_ARG, "unsupported row tuning (nt=%d, k=%d, layout=%d)", nt, k,
                     layout);
  g_row_override = Tuning1D{nt, k, layout};
  return WZN_OK;
}

int32_t wzn_get_row_tuning(int32_t nvar, int64_t n, int32_t* nt, int32_t* k, int32_t* layout) {
  g_err[0] = 0;
  if (!nt || !k || !layout) return set_error(WZN_ERR_ARG, "null output pointer");
  if (nvar != 1 && nvar != 3) return set_error(WZN_ERR_ARG, "nvar must be 1 or 3");
  const Tuning1D t = tuning_1d(nvar, n);
  *nt = t.nt;
  *k = t.k;
  *layout = t.layout;
  return WZN_OK;
}

size_t wzn_workspace_bytes(const wzn_params* p, int64_t nx, int64_t ny) {
  (void)p; (void)nx; (void)ny;
  return sizeof(unsigned long long) * WS_WORDS;
}

int32_t wzn_reconstruct(const wzn_params* p, const double* f, double* fhat, int64_t m,
                        void* stream) {
  g_err[0] = 0;
  int st = check_params(p, false, true);
  if (st) return st;
  if (m < 0 || m > ((int64_t)1 << 34)) return set_error(WZN_ERR_SIZE, "m out of range");
  if (m == 0) return WZN_OK;  // (empty arrays may be NULL)
  if (!f || !fhat) return set_error(WZN_ERR_ARG, "f or fhat is NULL");
  return reconstruct(p, f, fhat, m, (hipStream_t)stream);
}

int32_t wzn_rhs_1d(const wzn_params* p, const void* u, void* dudt, int64_t n, double dx,
                   void* ws, void* stream) {
  g_err[0] = 0;
  int st = check_1d(p, n, dx, ws, true);
  if (st) return st;
  if (!u || !dudt) return set_error(WZN_ERR_ARG, "u or dudt is NULL");
  if (u == dudt) return set_error(WZN_ERR_ARG, "u and dudt must not alias");
  Workspace w = make_workspace(ws);
  const int64_t nv = p->system == WZN_EULER ? 3 : 1;
  st = state_checked(rhs_1d(p, (const double*)u, (double*)dudt, n, dx, &w, (hipStream_t)stream),
                     p, u, n, (int)nv, false, true, &w, stream);
  return scanned(st, p, dudt, nv * n, false, &w, stream);
}

int32_t wzn_speed_max_1d(const wzn_params* p, const void* u, int64_t n, double* speed1,
                         void* ws, void* stream) {
  g_err[0] = 0;
  int st = check_1d(p, n, 1.0, ws);
  if (st) return st;
  if (p->system != WZN_EULER) return set_error(WZN_ERR_ARG, "1D Euler only");
  if (!u || !speed1) return set_error(WZN_ERR_ARG, "NULL array argument");
  Workspace w = make_workspace(ws);
  st = speed_max_1d(p, (const double*)u, n, speed1, &w, (hipStream_t)stream);
  return state_checked(st, p, u, n, 3, false, false, &w, stream);
}

int32_t wzn_rhs_1d_slab(const wzn_params* p, const void* u, const void* ghost_lo,
                        const void* ghost_hi, void* dudt, int64_t n, double dx,
                        const double* alpha, void* ws, void* stream) {
  g_err[0] = 0;
  int st = check_1d(p, n, dx, ws);
  if (st) return st;
  if (p->system != WZN_EULER) return set_error(WZN_ERR_ARG, "slabs are for 1D Euler");
  if (!u || !ghost_lo || !ghost_hi || !dudt || !alpha)
    return set_error(WZN_ERR_ARG, "NULL argument");
  if (u == dudt) return set_error(WZN_ERR_ARG, "u and dudt must not alias");
  Workspace w = make_workspace(ws);
  st = state_checked(rhs_1d_slab(p, (const double*)u, (const double*)ghost_lo,
                                 (const double*)ghost_hi, (double*)dudt, n, dx, alpha,
                                 (hipStream_t)stream),
                     p, u, n, 3, false, true, &w, stream);
  return scanned(st, p, dudt, 3 * n, false, &w, stream);
}

int32_t wzn_rk3_run_1d(const wzn_params* p, void* u, void* stage, int64_t n, double dx,
                       double cfl, int32_t nsteps, const double* dt_in, const double* alpha_in,
                       double* dt_out, double* alpha_out, void* ws, void* stream) {
  g_err[0] = 0;
  int st = check_1d(p, n, dx, ws, true);
  if (st) return st;
  if (!u || !stage) return set_error(WZN_ERR_ARG, "u or stage is NULL");
  if (nsteps < 0) return set_error(WZN_ERR_ARG, "nsteps < 0");
  if (!dt_in && !(cfl > 0.0)) return set_error(WZN_ERR_ARG, "cfl must be positive");
  Workspace w = make_workspace(ws);
  const int64_t nv = p->system == WZN_EULER ? 3 : 1;
  st = scanned(rk3_run_1d(p, (double*)u, (double*)stage, n, dx, cfl, nsteps, dt_in, alpha_in,
                          dt_out, alpha_out, &w, (hipStream_t)stream),
               p, u, nv * n, false, &w, stream);
  return state_checked(st, p, u, n, (int)nv, false, true, &w, stream);
}

int32_t wzn_rk3_step_1d(const wzn_params* p, void* u, void* stage, int64_t n, double dx,
                        double cfl, const double* dt_in, double* dt_out, void* ws,
                        void* stream) {
  return wzn_rk3_run_1d(p, u, stage, n, dx, cfl, 1, dt_in, nullptr, dt_out, nullptr, ws, stream);
}

int32_t wzn_rhs_1d_char(const wzn_params* p, const void* u, void* dudt, int64_t n, double dx,
                        const double* alpha3, void* ws, void* stream) {
  g_err[0] = 0;
  int st = check_1d(p, n, dx, ws);
  if (st) return st;
  if (p->system != WZN_EULER)
    return set_error(WZN_ERR_ARG, "characteristic fields exist for the Euler system only");
  if (!u || !dudt) return set_error(WZN_ERR_ARG, "u or dudt is NULL");
  if (u == dudt) return set_error(WZN_ERR_ARG, "u and dudt must not alias");
  Workspace w = make_workspace(ws);
  st = state_checked(rhs_1d_char(p, (const double*)u, (double*)dudt, n, dx, alpha3, &w,
                                 (hipStream_t)stream),
                     p, u, n, 3, false, false, &w, stream);
  return scanned(st, p, dudt, 3 * n, false, &w, stream);
}

int32_t wzn_rk3_run_1d_char(const wzn_params* p, void* u, void* stage, int64_t n, double dx,
                            double cfl, int32_t nsteps, const double* dt_in,
                            const double* alpha_in, double* dt_out, double* alpha_out, void* ws,
                            void* stream) {
  g_err[0] = 0;
  int st = check_1d(p, n, dx, ws);
  if (st) return st;
  if (p->system != WZN_EULER)
    return set_error(WZN_ERR_ARG, "characteristic fields exist for the Euler system only");
  if (!u || !stage) return set_error(WZN_ERR_ARG, "u or stage is NULL");
  if (nsteps < 0) return set_error(WZN_ERR_ARG, "nsteps < 0");
  if (!dt_in && !(cfl > 0.0)) return set_error(WZN_ERR_ARG, "cfl must be positive");
  Workspace w = make_workspace(ws);
  st = scanned(rk3_run_1d_char(p, (double*)u, (double*)stage, n, dx, cfl, nsteps, dt_in,
                               alpha_in, dt_out, alpha_out, &w, (hipStream_t)stream),
               p, u, 3 * n, false, &w, stream);
  return state_checked(st, p, u, n, 3, false, false, &w, stream);
}

int32_t wzn_rhs_2d(const wzn_params* p, const void* u, void* dudt, int64_t nx, int64_t ny,
                   double dx, double dy, void* ws, void* stream) {
  g_err[0] = 0;
  int st = check_2d(p, nx, ny, dx, dy, ws);
  if (st) return st;
  if (!u || !dudt) return set_error(WZN_ERR_ARG, "u or dudt is NULL");
  if (u == dudt) return set_error(WZN_ERR_ARG, "u and dudt must not alias");
  Workspace w = make_workspace(ws);
  const bool f32 = p->dtype == WZN_FP32;
  st = f32 ? rhs_2d_t<float>(p, (const float*)u, (float*)dudt, nx, ny, dx, dy, &w,
                             (hipStream_t)stream)
           : rhs_2d_t<double>(p, (const double*)u, (double*)dudt, nx, ny, dx, dy, &w,
                              (hipStream_t)stream);
  st = state_checked(st, p, u, nx * ny, 4, f32, true, &w, stream);
  return scanned(st, p, dudt, 4 * nx * ny, f32, &w, stream);
}

int32_t wzn_rhs_2d_strip(const wzn_params* p, const void* u, const void* ghost_lo,
                         const void* ghost_hi, void* dudt, int64_t nx, int64_t ny, double dx,
                         double dy, const double* alpha2, void* ws, void* stream) {
  g_err[0] = 0;
  int st = check_2d(p, nx, ny, dx, dy, ws);
  if (st) return st;
  if (!u || !ghost_lo || !ghost_hi || !dudt)
    return set_error(WZN_ERR_ARG, "NULL array argument");
  if (u == dudt) return set_error(WZN_ERR_ARG, "u and dudt must not alias");
  if (p->flux_split == WZN_SPLIT_LF && !alpha2)
    return set_error(WZN_ERR_ARG, "the Lax-Friedrichs split of a strip needs the global alphas");
  Workspace w = make_workspace(ws);
  const bool f32 = p->dtype == WZN_FP32;
  st = f32 ? rhs_2d_strip_t<float>(p, (const float*)u, (const float*)ghost_lo,
                                   (const float*)ghost_hi, (float*)dudt, nx, ny, dx, dy, alpha2,
                                   (hipStream_t)stream)
           : rhs_2d_strip_t<double>(p, (const double*)u, (const double*)ghost_lo,
                                    (const double*)ghost_hi, (double*)dudt, nx, ny, dx, dy,
                                    alpha2, (hipStream_t)stream);
  st = state_checked(st, p, u, nx * ny, 4, f32, true, &w, stream);
  return scanned(st, p, dudt, 4 * nx * ny, f32, &w, stream);
}

int32_t wzn_speed_max_2d(const wzn_params* p, const void* u, int64_t nx, int64_t ny,
                         double* speed2, void* ws, void* stream) {
  g_err[0] = 0;
  int st = check_2d(p, nx, ny, 1.0, 1.0, ws);
  if (st) return st;
  if (!u || !speed2) return set_error(WZN_ERR_ARG, "NULL array argument");
  Workspace w = make_workspace(ws);
  const bool f32 = p->dtype == WZN_FP32;
  st = f32 ? speed_max_2d_t<float>(p, (const float*)u, nx, ny, speed2, &w, (hipStream_t)stream)
           : speed_max_2d_t<double>(p, (const double*)u, nx, ny, speed2, &w,
                                    (hipStream_t)stream);
  return state_checked(st, p, u, nx * ny, 4, f32, false, &w, stream);
}

int32_t wzn_rk3_run_2d(const wzn_params* p, void* u, void* stage, int64_t nx, int64_t ny,
                       double dx, double dy, double cfl, int32_t nsteps, const double* dt_in,
                       double* dt_out, void* ws, void* stream) {
  g_err[0] = 0;
  int st = check_2d(p, nx, ny, dx, dy, ws);
  if (st) return st;
  if (!u || !stage) return set_error(WZN_ERR_ARG, "u or stage is NULL");
  if (nsteps < 0) return set_error(WZN_ERR_ARG, "nsteps < 0");
  if (!dt_in && !(cfl > 0.0)) return set_error(WZN_ERR_ARG, "cfl must be positive");
  Workspace w = make_workspace(ws);
  const bool f32 = p->dtype == WZN_FP32;
  st = f32 ? rk3_run_2d_t<float>(p, (float*)u, (float*)stage, nx, ny, dx, dy, cfl, nsteps,
                                 dt_in, dt_out, &w, (hipStream_t)stream)
           : rk3_run_2d_t<double>(p, (double*)u, (double*)stage, nx, ny, dx, dy, cfl, nsteps,
                                  dt_in, dt_out, &w, (hipStream_t)stream);
  st = scanned(st, p, u, 4 * nx * ny, f32, &w, stream);
  return state_checked(st, p, u, nx * ny, 4, f32, true, &w, stream);
}

int64_t wzn_char2d_work_doubles(int64_t nx, int64_t ny) {
  return nx > 0 && ny > 0 ? 4 * nx * ny : 0;
}

static int check_char2d(const wzn_params* p, int64_t nx, int64_t ny, double dx, double dy,
                        void* ws, const void* work) {
  int st = check_2d(p, nx, ny, dx, dy, ws);
  if (st) return st;
  if (p->dtype != WZN_FP64)
    return set_error(WZN_ERR_DTYPE, "characteristic fields run in fp64 only");
  if (p->flux_split != WZN_SPLIT_LF)
    return set_error(WZN_ERR_UNSUPPORTED, "characteristic fields use the Lax-Friedrichs split");
  if (p->weights != WZN_WEIGHTS_ZN)
    return set_error(WZN_ERR_UNSUPPORTED, "characteristic fields run the WENO-ZN weights");
  if (!work) return set_error(WZN_ERR_ARG, "work is NULL");
  return WZN_OK;
}

int32_t wzn_rhs_2d_char(const wzn_params* p, const void* u, void* dudt, void* work, int64_t nx,
                        int64_t ny, double dx, double dy, const double* alpha8, void* ws,
                        void* stream) {
  g_err[0] = 0;
  int st = check_char2d(p, nx, ny, dx, dy, ws, work);
  if (st) return st;
  if (!u || !dudt) return set_error(WZN_ERR_ARG, "u or dudt is NULL");
  if (u == dudt || work == u || work == dudt)
    return set_error(WZN_ERR_ARG, "u, dudt and work must not alias");
  Workspace w = make_workspace(ws);
  st = state_checked(rhs_2d_char(p, (const double*)u, (double*)dudt, (double*)work, nx, ny, dx,
                                 dy, alpha8, &w, (hipStream_t)stream),
                     p, u, nx * ny, 4, false, false, &w, stream);
  return scanned(st, p, dudt, 4 * nx * ny, false, &w, stream);
}

int32_t wzn_rk3_run_2d_char(const wzn_params* p, void* u, void* stage, void* work, int64_t nx,
                            int64_t ny, double dx, double dy, double cfl, int32_t nsteps,
                            const double* dt_in, double* dt_out, void* ws, void* stream) {
  g_err[0] = 0;
  int st = check_char2d(p, nx, ny, dx, dy, ws, work);
  if (st) return st;
  if (!u || !stage) return set_error(WZN_ERR_ARG, "u or stage is NULL");
  if (work == u || work == stage || stage == u)
    return set_error(WZN_ERR_ARG, "u, stage and work must not alias");
  if (nsteps < 0) return set_error(WZN_ERR_ARG, "nsteps < 0");
  if (!dt_in && !(cfl > 0.0)) return set_error(WZN_ERR_ARG, "cfl must be positive");
  Workspace w = make_workspace(ws);
  st = scanned(rk3_run_2d_char(p, (double*)u, (double*)stage, (double*)work, nx, ny, dx, dy,
                               cfl, nsteps, dt_in, dt_out, &w, (hipStream_t)stream),
               p, u, 4 * nx * ny, false, &w, stream);
  return state_checked(st, p, u, nx * ny, 4, false, false, &w, stream);
}

int32_t wzn_rk3_step_2d(const wzn_params* p, void* u, void* stage, int64_t nx, int64_t ny,
                        double dx, double dy, double cfl, const double* dt_in, double* dt_out,
                        void* ws, void* stream) {
  return wzn_rk3_run_2d(p, u, stage, nx, ny, dx, dy, cfl, 1, dt_in, dt_out, ws, stream);
}

int32_t wzn_batched_rk3_run_1d(const wzn_params* p, void* u, void* stage, int64_t total,
                               const int64_t* offsets, const double* dx, const int32_t* order,
                               int32_t batch, int32_t nsteps, double cfl,
                               const wzn_batch_tuning* tuning, double* dt_out, void* ws,
                               void* stream) {
  g_err[0] = 0;
  int st = check_1d(p, total, 1.0, ws);
  if (st) return st;
  if (p->system != WZN_EULER) return set_error(WZN_ERR_ARG, "batched runs are 1D Euler only");
  if (p->lf_alpha_x >= 0.0)
    return set_error(WZN_ERR_UNSUPPORTED, "batched runs always reduce alpha (lf_alpha_x < 0)");
  if (!u || !stage || !offsets || !dx) return set_error(WZN_ERR_ARG, "NULL array argument");
  if (batch < 1) return set_error(WZN_ERR_ARG, "batch < 1");
  if (nsteps < 0) return set_error(WZN_ERR_ARG, "nsteps < 0");
  if (!(cfl > 0.0)) return set_error(WZN_ERR_ARG, "cfl must be positive");
  if (tuning) {
    const int nt = tuning->nt, k = tuning->k;
    const bool ok = (nt == 64 && (k == 2 || k == 4)) || (nt == 128 && (k == 2 || k == 4)) ||
                    (nt == 256 && (k == 1 || k == 2 || k == 4));
    if (!ok) return set_error(WZN_ERR_ARG, "unsupported batched tuning (nt=%d, k=%d)", nt, k);
  }
  Workspace w = make_workspace(ws);
  st = scanned(batched_rk3_run_1d(p, (double*)u, (double*)stage, total, offsets, dx, order,
                                  batch, nsteps, cfl, tuning, dt_out, &w, (hipStream_t)stream),
               p, u, 3 * total, false, &w, stream);
  return state_checked(st, p, u, total, 3, false, true, &w, stream);
}

int32_t wzn_rhs_1d_vjp(const wzn_params* p, const void* u, const void* mu, void* out, int64_t n,
                       double dx, void* ws, void* stream) {
  g_err[0] = 0;
  int st = check_1d(p, n, dx, ws);
  if (st) return st;
  if (p->system != WZN_EULER) return set_error(WZN_ERR_ARG, "the adjoint is for 1D Euler");
  if (!u || !mu || !out) return set_error(WZN_ERR_ARG, "NULL array argument");
  if (out == u || out == mu) return set_error(WZN_ERR_ARG, "out must not alias u or mu");
  Workspace w = make_workspace(ws);
  st = state_checked(rhs_1d_vjp(p, (const double*)u, (const double*)mu, (double*)out, n, dx, &w,
                                (hipStream_t)stream),
                     p, u, n, 3, false, true, &w, stream);
  return scanned(st, p, out, 3 * n, false, &w, stream);
}

int32_t wzn_rk3_step_1d_vjp(const wzn_params* p, const void* stages, const void* lam_next,
                            void* lam_prev, void* scratch, int64_t n, double dx,
                            const double* dt, const double* alpha3, void* ws, void* stream) {
  g_err[0] = 0;
  int st = check_1d(p, n, dx, ws);
  if (st) return st;
  if (p->system != WZN_EULER) return set_error(WZN_ERR_ARG, "the adjoint is for 1D Euler");
  if (!stages || !lam_next || !lam_prev || !scratch || !dt || !alpha3)
    return set_error(WZN_ERR_ARG, "NULL argument");
  if (lam_prev == lam_next || lam_prev == stages || lam_prev == scratch)
    return set_error(WZN_ERR_ARG, "lam_prev must not alias the other arrays");
  Workspace w = make_workspace(ws);
  st = rk3_step_1d_vjp(p, (const double*)stages, (const double*)lam_next, (double*)lam_prev,
                       (double*)scratch, n, dx, dt, alpha3, &w, (hipStream_t)stream);
  for (int k = 0; k < 3; ++k)
    st = state_checked(st, p, (const double*)stages + (int64_t)k * 3 * n, n, 3, false, true, &w,
                       stream);
  return scanned(st, p, lam_prev, 3 * n, false, &w, stream);
}

int64_t wzn_rk3_adjoint_1d_work_doubles(int64_t n, int32_t ckpt_every) {
  if (n < 1 || ckpt_every < 1) return 0;
  return ((int64_t)ckpt_every * 3 + 3) * 3 * n + 3 * n;
}

int32_t wzn_rk3_adjoint_1d(const wzn_params* p, const void* ckpts, int32_t nsteps,
                           int32_t ckpt_every, const double* dts, const double* alphas,
                           void* lam, void* work, int64_t n, double dx, void* ws, void* stream) {
  g_err[0] = 0;
  int st = check_1d(p, n, dx, ws);
  if (st) return st;
  if (p->system != WZN_EULER) return set_error(WZN_ERR_ARG, "the adjoint is for 1D Euler");
  if (!ckpts || !dts || !alphas || !lam || !work) return set_error(WZN_ERR_ARG, "NULL argument");
  if (nsteps < 0 || ckpt_every < 1) return set_error(WZN_ERR_ARG, "bad nsteps / ckpt_every");
  Workspace w = make_workspace(ws);
  st = rk3_adjoint_1d(p, (const double*)ckpts, nsteps, ckpt_every, dts, alphas, (double*)lam,
                      (double*)work, n, dx, &w, (hipStream_t)stream);
  const int32_t nseg = (nsteps + ckpt_every - 1) / ckpt_every;
  for (int32_t k = 0; k < nseg; ++k)
    st = state_checked(st, p, (const double*)ckpts + (int64_t)k * 3 * n, n, 3, false, true, &w,
                       stream);
  return scanned(st, p, lam, 3 * n, false, &w, stream);
}

}  // extern "C"
