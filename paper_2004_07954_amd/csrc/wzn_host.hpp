// Host-side helpers shared by the translation units of libwenozn: error reporting,
// workspace layout and launch tuning.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wenozn.h"

namespace wzn {

// Layout of the caller's device workspace (64-bit words).
struct Workspace {
  unsigned long long* speed;    // [3] ring of max(|u|+c) slots (x direction)
  unsigned long long* speed_y;  // [3] ring of max(|v|+c) slots (y direction)
  double* dt;                   // [1] dt of the current step
  unsigned long long* counter;  // [1] work-queue counter (batched launch)
  unsigned long long* char_speed;  // [3][3] ring of per-field alpha triples (characteristic)
  unsigned long long* scratch;  // [WS_SCRATCH_WORDS] spare words
};
constexpr int WS_WORDS = 512;  // 4 KiB
constexpr int WS_SCRATCH_WORDS = WS_WORDS - 32;

inline Workspace make_workspace(void* ws) {
  unsigned long long* w = (unsigned long long*)ws;
  Workspace s;
  s.speed = w;
  s.speed_y = w + 3;
  s.dt = (double*)(w + 6);
  s.counter = w + 7;
  s.char_speed = w + 16;
  s.scratch = w + 32;
  return s;
}

struct Tuning1D {
  int nt;      // threads per workgroup
  int k;       // consecutive cells (interfaces) per thread
  int layout;  // ROW_LDS_TILE: both signs of the split flux staged in LDS at once;
               // ROW_LDS_SPLIT: one sign at a time (half the LDS)
};
enum { ROW_LDS_TILE = 0, ROW_LDS_SPLIT = 1 };
Tuning1D tuning_1d(int nv, int64_t n);
Tuning1D row_override();  // the wzn_set_row_tuning override ({0, 0, 0} when unset)

int set_error(int code, const char* fmt, ...);
int check_launch(const char* what);
int launch_zero_words(unsigned long long* p, int count, hipStream_t s);
int launch_fill_double(double* p, double v, hipStream_t s);

template <typename T>
int launch_speed_max(const T* u, int64_t n, int nv, double gamma, unsigned long long* slot,
                     unsigned long long* slot_y, hipStream_t s);

template <typename T>
int rhs_2d_t(const wzn_params* p, const T* u, T* dudt, int64_t nx, int64_t ny, double dx,
             double dy, Workspace* ws, hipStream_t s);
template <typename T>
int rhs_2d_strip_t(const wzn_params* p, const T* u, const T* ghost_lo, const T* ghost_hi,
                   T* dudt, int64_t nx, int64_t ny, double dx, double dy, const double* alpha2,
                   hipStream_t s);
template <typename T>
int speed_max_2d_t(const wzn_params* p, const T* u, int64_t nx, int64_t ny, double* out,
                   Workspace* ws, hipStream_t s);
template <typename T>
int rk3_run_2d_t(const wzn_params* p, T* u, T* stage, int64_t nx, int64_t ny, double dx,
                 double dy, double cfl, int32_t nsteps, const double* dt_in, double* dt_out,
                 Workspace* ws, hipStream_t s);

int batched_rk3_run_1d(const wzn_params* p, double* u, double* stage, int64_t total,
                       const int64_t* offsets, const double* dx, const int32_t* order,
                       int32_t batch, int32_t nsteps, double cfl, const wzn_batch_tuning* tn,
                       double* dt_out, Workspace* ws, hipStream_t s);

int rhs_1d_char(const wzn_params* p, const double* u, double* dudt, int64_t n, double dx,
                const double* alpha3, Workspace* ws, hipStream_t s);
int rk3_run_1d_char(const wzn_params* p, double* u, double* stage, int64_t n, double dx,
                    double cfl, int32_t nsteps, const double* dt_in, const double* alpha_in,
                    double* dt_out, double* alpha_out, Workspace* ws, hipStream_t s);

int rhs_2d_char(const wzn_params* p, const double* u, double* dudt, double* work, int64_t nx,
                int64_t ny, double dx, double dy, const double* alpha8, Workspace* ws,
                hipStream_t s);
int rk3_run_2d_char(const wzn_params* p, double* u, double* stage, double* work, int64_t nx,
                    int64_t ny, double dx, double dy, double cfl, int32_t nsteps,
                    const double* dt_in, double* dt_out, Workspace* ws, hipStream_t s);

int rhs_1d_vjp(const wzn_params* p, const double* u, const double* mu, double* out, int64_t n,
               double dx, Workspace* ws, hipStream_t s);
int rk3_step_1d_vjp(const wzn_params* p, const double* stages, const double* lam_next,
                    double* lam_prev, double* scratch, int64_t n, double dx, const double* dt,
                    const double* alpha3, Workspace* ws, hipStream_t s);

int rk3_adjoint_1d(const wzn_params* p, const double* ckpts, int32_t nsteps, int32_t ckpt_every,
                   const double* dts, const double* alphas, double* lam, double* work,
                   int64_t n, double dx, Workspace* ws, hipStream_t s);

int rhs_1d(const wzn_params* p, const double* u, double* dudt, int64_t n, double dx,
           Workspace* ws, hipStream_t s);
int reconstruct(const wzn_params* p, const double* f, double* fhat, int64_t m, hipStream_t s);
int rhs_1d_slab(const wzn_params* p, const double* u, const double* ghost_lo,
                const double* ghost_hi, double* dudt, int64_t n, double dx, const double* alpha,
                hipStream_t s);
int speed_max_1d(const wzn_params* p, const double* u, int64_t n, double* out, Workspace* ws,
                 hipStream_t s);
// NaN / Inf scan of an output (the debug_nonfinite mode): synchronises s; WZN_ERR_NONFINITE
// if any value of x[0 .. count) is not finite
int debug_nonfinite_scan(const void* x, int64_t count, bool f32, Workspace* ws, hipStream_t s);
// The debug mode's scan of a state u of N cells and nv components (1: advection, 3: 1D Euler,
// 4: 2D Euler): WZN_ERR_NONPHYSICAL if a cell has rho <= 0 or p <= 0, and (check_range)
// WZN_ERR_RANGE if the split fluxes F +- alpha U may exceed the weights' range (1e26 in fp64,
// 1e17 in fp32).  Does nothing unless p->debug_nonfinite; synchronises s.
int debug_state_scan(const wzn_params* p, const void* u, int64_t N, int nv, bool f32,
                     bool check_range, Workspace* ws, hipStream_t s);
int rk3_run_1d(const wzn_params* p, double* u, double* stage, int64_t n, double dx, double cfl,
               int32_t nsteps, const double* dt_in, const double* alpha_in, double* dt_out,
               double* alpha_out, Workspace* ws, hipStream_t s);

}  // namespace wzn
