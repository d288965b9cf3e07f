// Host side of the 1D path: the right-hand side and the TVD-RK3 run, enqueued as row-kernel
// launches with the global Lax-Friedrichs alpha / CFL dt carried between kernels in a ring of
// device slots (no host synchronisation, so a run can be captured in a HIP graph).
//
// Slot protocol for a run: kernel number s (s = 0, 1, 2, ... over all stages of all steps)
// reads the speed slot ring[s % 3] (alpha of its input, and dt for the first stage of a
// step), atomically maxes the wave speed of its output into ring[(s + 1) % 3], and clears
// ring[(s + 2) % 3], whose last reader was kernel s - 1.
#include <hip/hip_runtime.h>

#include "wzn_device.hpp"
#include "wzn_host.hpp"
#include "wzn_rows.hpp"
#include "wzn_tile.hpp"

namespace wzn {

// max over cells of the largest wave speed into *slot (slot must be zero beforehand):
// |u| + c for 1D Euler; (|u| + c, |v| + c) into (slot, slot_y) for 2D Euler.  A grid-stride
// loop that takes four cells per thread and iteration, their loads issued together.
template <int NV, typename T>
__device__ __forceinline__ void speed_of_cell(const T (&U)[NV], double gamma, double& sx,
                                              double& sy) {
  if constexpr (NV == 3) {
    const double D[3] = {double(U[0]), double(U[1]), double(U[2])};
    sx = fmax(sx, wave_speed_1d<SYS_EULER1>(D, 0.0, gamma));
  } else {
    double a, b;
    wave_speeds_2d(U[0], U[1], U[2], U[3], gamma, a, b);
    sx = fmax(sx, a);
    sy = fmax(sy, b);
  }
}

template <int NV, typename T>
__global__ __launch_bounds__(256) void speed_max_kernel(const T* __restrict__ u, int64_t n,
                                                        double gamma, unsigned long long* slot,
                                                        unsigned long long* slot_y) {
  constexpr int UNR = 4;
  double sx = 0.0, sy = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + (UNR - 1) * stride < n; i += UNR * stride) {
    T U[UNR][NV];
#pragma unroll
    for (int q = 0; q < UNR; ++q)
#pragma unroll
      for (int c = 0; c < NV; ++c) U[q][c] = u[c * n + i + q * stride];
#pragma unroll
    for (int q = 0; q < UNR; ++q) speed_of_cell<NV, T>(U[q], gamma, sx, sy);
  }
  for (; i < n; i += stride) {
    T U[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) U[c] = u[c * n + i];
    speed_of_cell<NV, T>(U, gamma, sx, sy);
  }
  __shared__ double red[2][4];
  sx = wave_max(sx);
  sy = wave_max(sy);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sx;
    red[1][threadIdx.x >> 6] = sy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomic_max_pos(slot, fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3])));
    if (NV == 4)
      atomic_max_pos(slot_y, fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3])));
  }
}

__global__ void zero_words_kernel(unsigned long long* p, int count) {
  const int i = threadIdx.x;
  if (i < count) p[i] = 0ull;
}

int launch_zero_words(unsigned long long* p, int count, hipStream_t s) {
  if (count > 64) return set_error(WZN_ERR_ARG, "zero_words: count > 64");
  hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, p, count);
  return check_launch("zero_words_kernel");
}

template <typename T>
int launch_speed_max(const T* u, int64_t n, int nv, double gamma, unsigned long long* slot,
                     unsigned long long* slot_y, hipStream_t s) {
  // at most 512 workgroups: every workgroup ends with one atomic on the same word, and at
  // 2048 of them finishing together those atomics cost more than the reduction itself
  int64_t blocks = (n + 255) / 256;
  if (blocks > 512) blocks = 512;
  if (nv == 3)
    hipLaunchKernelGGL((speed_max_kernel<3, T>), dim3((unsigned)blocks), dim3(256), 0, s, u, n,
                       gamma, slot, slot_y);
  else
    hipLaunchKernelGGL((speed_max_kernel<4, T>), dim3((unsigned)blocks), dim3(256), 0, s, u, n,
                       gamma, slot, slot_y);
  return check_launch("speed_max_kernel");
}
template int launch_speed_max<double>(const double*, int64_t, int, double, unsigned long long*,
                                      unsigned long long*, hipStream_t);
template int launch_speed_max<float>(const float*, int64_t, int, double, unsigned long long*,
                                     unsigned long long*, hipStream_t);

static RowArgs<double> base_args(const wzn_params* p, int64_t n, double dx) {
  RowArgs<double> a{};
  a.n = n;
  a.plane = n;
  a.row_stride = 0;
  a.dx = dx;
  a.bc = p->bc_x;
  a.adv = p->adv_speed;
  a.gamma = p->gamma;
  a.eps_s = 16.0 * p->eps;
  a.A = p->A;
  a.weights = p->weights;
  return a;
}

static int sys_of(const wzn_params* p) { return p->system == WZN_EULER ? SYS_EULER1 : SYS_ADV; }

int rhs_1d(const wzn_params* p, const double* u, double* dudt, int64_t n, double dx, Workspace* ws,
           hipStream_t s) {
  const int nv = p->system == WZN_EULER ? 3 : 1;
  RowArgs<double> a = base_args(p, n, dx);
  a.uin = u;
  a.out = dudt;
  a.mode = MODE_RHS;
  if (p->lf_alpha_x >= 0.0) {
    a.alpha_const = p->lf_alpha_x;
  } else if (nv == 1) {
    a.alpha_const = __builtin_fabs(p->adv_speed);
  } else {
    int st = launch_zero_words(ws->speed, 1, s);
    if (st) return st;
    st = launch_speed_max<double>(u, n, 3, p->gamma, ws->speed, nullptr, s);
    if (st) return st;
    a.alpha_slot = ws->speed;
  }
  return launch_rows(a, sys_of(p), 1, tuning_1d(nv, n), s);
}

// Right-hand side of a slab of n cells of a longer 1D Euler row (one GPU's share of a slab
// decomposition): its three cells on each side from ghost_lo / ghost_hi ([3][3], component
// major), and the caller's alpha (the maximum over the whole row: a per-slab alpha would change
// the scheme).
int rhs_1d_slab(const wzn_params* p, const double* u, const double* ghost_lo,
                const double* ghost_hi, double* dudt, int64_t n, double dx, const double* alpha,
                hipStream_t s) {
  RowArgs<double> a = base_args(p, n, dx);
  a.uin = u;
  a.out = dudt;
  a.mode = MODE_RHS;
  a.alpha_arr = alpha;
  a.ghost_lo = ghost_lo;
  a.ghost_hi = ghost_hi;
  return launch_rows(a, SYS_EULER1, 1, tuning_1d(3, n), s);
}

// max over the cells of u [3][n] of |u| + c into *out (device double)
__global__ void slot_to_double_kernel(const unsigned long long* slot, double* out) {
  if (threadIdx.x == 0) out[0] = slot_value(slot);
}

int speed_max_1d(const wzn_params* p, const double* u, int64_t n, double* out, Workspace* ws,
                 hipStream_t s) {
  int st = launch_zero_words(ws->speed, 1, s);
  if (st) return st;
  st = launch_speed_max<double>(u, n, 3, p->gamma, ws->speed, nullptr, s);
  if (st) return st;
  hipLaunchKernelGGL(slot_to_double_kernel, dim3(1), dim3(64), 0, s, ws->speed, out);
  return check_launch("slot_to_double_kernel");
}

// One reconstruction per thread from five point values (structure of arrays [5][m]).  The
// window carries its indicators scaled by 4, so eps enters as 4 eps (see wzn_device.hpp).
template <int WT>
__global__ __launch_bounds__(256) void reconstruct_kernel(const double* __restrict__ f,
                                                          double* __restrict__ fhat, int64_t m,
                                                          double eps_s, double Aq) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * 256) {
    double v[5], h[1];
#pragma unroll
    for (int j = 0; j < 5; ++j) v[j] = f[j * m + i];
    wzn_window<1, WT>(v, h, eps_s, Aq);
    fhat[i] = h[0];
  }
}

int reconstruct(const wzn_params* p, const double* f, double* fhat, int64_t m, hipStream_t s) {
  int64_t blocks = (m + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (p->weights == WZN_WEIGHTS_Z)
    hipLaunchKernelGGL((reconstruct_kernel<WEIGHTS_Z>), dim3((unsigned)blocks), dim3(256), 0, s,
                       f, fhat, m, 4.0 * p->eps, 0.25 * p->A);
  else
    hipLaunchKernelGGL((reconstruct_kernel<WEIGHTS_ZN>), dim3((unsigned)blocks), dim3(256), 0, s,
                       f, fhat, m, 4.0 * p->eps, 0.25 * p->A);
  return check_launch("reconstruct_kernel");
}

// Count of non-finite values of x[0 .. count) into flag[0] and the largest index + 1 of one into
// flag[1] (both zero beforehand).
template <typename T>
__global__ __launch_bounds__(256) void nonfinite_scan_kernel(const T* __restrict__ x, int64_t count,
                                                             unsigned long long* flag) {
  unsigned long long bad = 0, last = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256) {
    if (!__builtin_isfinite(double(x[i]))) {
      ++bad;
      last = (unsigned long long)i + 1;
    }
  }
  if (bad) {
    atomicAdd(&flag[0], bad);
    atomicMax(&flag[1], last);
  }
}

int debug_nonfinite_scan(const void* x, int64_t count, bool f32, Workspace* ws, hipStream_t s) {
  unsigned long long* flag = ws->scratch;
  int st = launch_zero_words(flag, 2, s);
  if (st) return st;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  if (f32)
    hipLaunchKernelGGL((nonfinite_scan_kernel<float>), dim3((unsigned)blocks), dim3(256), 0, s,
                       (const float*)x, count, flag);
  else
    hipLaunchKernelGGL((nonfinite_scan_kernel<double>), dim3((unsigned)blocks), dim3(256), 0, s,
                       (const double*)x, count, flag);
  st = check_launch("nonfinite_scan_kernel");
  if (st) return st;
  unsigned long long host[2] = {0, 0};
  if (hipMemcpyAsync(host, flag, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(WZN_ERR_HIP, "debug scan: copy of the flag failed");
  if (host[0])
    return set_error(WZN_ERR_NONFINITE, "%llu non-finite output values (one at element %lld)",
                     host[0], (long long)host[1] - 1);
  return WZN_OK;
}

// The debug mode's scan of a state (the input of a right-hand side, or the result of a run):
// the count of cells with rho <= 0 or p <= 0 (or not finite) and the largest index + 1 of one,
// and, over the other cells, the maxima from which the host bounds the split fluxes the
// reconstruction sees.  Words of out (zero beforehand; maxima as bit patterns of non-negative
// doubles): [0] count, [1] last index + 1, [2 + c] max |F_c|, [6 + c] max |G_c| (2D),
// [10 + c] max |U_c|, [14] max |u| + c, [15] max |v| + c.
constexpr int STATE_SCAN_WORDS = 16;

template <int NV, typename T>
__global__ __launch_bounds__(256) void state_scan_kernel(const T* __restrict__ u, int64_t N,
                                                         double gamma, double adv,
                                                         unsigned long long* out) {
  unsigned long long bad = 0, last = 0;
  double mF[4] = {0.0, 0.0, 0.0, 0.0}, mG[4] = {0.0, 0.0, 0.0, 0.0};
  double mU[4] = {0.0, 0.0, 0.0, 0.0}, sx = 0.0, sy = 0.0;
  const double gm1 = gamma - 1.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256) {
    double U[4] = {0.0, 0.0, 0.0, 0.0}, F[4] = {0.0, 0.0, 0.0, 0.0}, G[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < NV; ++c) U[c] = double(u[c * N + i]);
    bool ok;
    if constexpr (NV == 1) {
      F[0] = adv * U[0];
      ok = __builtin_isfinite(U[0]);
    } else if constexpr (NV == 3) {
      const double v = U[1] / U[0];
      const double p = gm1 * (U[2] - 0.5 * U[1] * v);
      F[0] = U[1];
      F[1] = U[1] * v + p;
      F[2] = v * (U[2] + p);
      ok = U[0] > 0.0 && p > 0.0 && __builtin_isfinite(U[0] + U[1] + U[2]);
      if (ok) sx = fmax(sx, __builtin_fabs(v) + sqrt(gamma * p / U[0]));
    } else {
      const double vx = U[1] / U[0], vy = U[2] / U[0];
      const double p = gm1 * (U[3] - 0.5 * (U[1] * vx + U[2] * vy));
      F[0] = U[1];
      F[1] = U[1] * vx + p;
      F[2] = U[2] * vx;
      F[3] = vx * (U[3] + p);
      G[0] = U[2];
      G[1] = U[1] * vy;
      G[2] = U[2] * vy + p;
      G[3] = vy * (U[3] + p);
      ok = U[0] > 0.0 && p > 0.0 && __builtin_isfinite(U[0] + U[1] + U[2] + U[3]);
      if (ok) {
        const double c = sqrt(gamma * p / U[0]);
        sx = fmax(sx, __builtin_fabs(vx) + c);
        sy = fmax(sy, __builtin_fabs(vy) + c);
      }
    }
    if (!ok) {
      ++bad;
      last = (unsigned long long)i + 1;
      continue;
    }
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      mF[c] = fmax(mF[c], __builtin_fabs(F[c]));
      mG[c] = fmax(mG[c], __builtin_fabs(G[c]));
      mU[c] = fmax(mU[c], __builtin_fabs(U[c]));
    }
  }
  if (bad) {
    atomicAdd(&out[0], bad);
    atomicMax(&out[1], last);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    mF[c] = wave_max(mF[c]);
    mG[c] = wave_max(mG[c]);
    mU[c] = wave_max(mU[c]);
  }
  sx = wave_max(sx);
  sy = wave_max(sy);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      atomic_max_pos(&out[2 + c], mF[c]);
      atomic_max_pos(&out[6 + c], mG[c]);
      atomic_max_pos(&out[10 + c], mU[c]);
    }
    atomic_max_pos(&out[14], sx);
    atomic_max_pos(&out[15], sy);
  }
}

int debug_state_scan(const wzn_params* p, const void* u, int64_t N, int nv, bool f32,
                     bool check_range, Workspace* ws, hipStream_t s) {
  if (!p->debug_nonfinite) return WZN_OK;
  unsigned long long* w = ws->scratch + 8;
  int st = launch_zero_words(w, STATE_SCAN_WORDS, s);
  if (st) return st;
  int64_t blocks = (N + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  const dim3 g((unsigned)blocks), b(256);
  if (nv == 1) {
    hipLaunchKernelGGL((state_scan_kernel<1, double>), g, b, 0, s, (const double*)u, N,
                       p->gamma, p->adv_speed, w);
  } else if (nv == 3) {
    hipLaunchKernelGGL((state_scan_kernel<3, double>), g, b, 0, s, (const double*)u, N,
                       p->gamma, 0.0, w);
  } else if (f32) {
    hipLaunchKernelGGL((state_scan_kernel<4, float>), g, b, 0, s, (const float*)u, N, p->gamma,
                       0.0, w);
  } else {
    hipLaunchKernelGGL((state_scan_kernel<4, double>), g, b, 0, s, (const double*)u, N,
                       p->gamma, 0.0, w);
  }
  st = check_launch("state_scan_kernel");
  if (st) return st;
  unsigned long long h[STATE_SCAN_WORDS];
  if (hipMemcpyAsync(h, w, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(WZN_ERR_HIP, "debug scan: copy of the state scan failed");
  if (h[0])
    return set_error(WZN_ERR_NONPHYSICAL,
                     "%llu cells with rho <= 0 or p <= 0 or a non-finite value (one at cell %lld)",
                     h[0], (long long)h[1] - 1);
  if (!check_range) return WZN_OK;
  double v[STATE_SCAN_WORDS];
  for (int k = 2; k < STATE_SCAN_WORDS; ++k) v[k] = __builtin_bit_cast(double, h[k]);
  // |F +- alpha U| <= |F| + alpha |U|: the Lax-Friedrichs alpha is the frozen one or the
  // state's largest wave speed, which also bounds the Steger-Warming split (its
  // eigenvalues are at most |u| + c)
  const bool adv = nv == 1;
  double ax = p->lf_alpha_x >= 0.0 ? p->lf_alpha_x : (adv ? __builtin_fabs(p->adv_speed) : v[14]);
  double ay = p->lf_alpha_y >= 0.0 ? p->lf_alpha_y : v[15];
  if (nv == 4 && p->flux_split == WZN_SPLIT_SW) {
    ax = v[14];
    ay = v[15];
  }
  double bound = 0.0;
  for (int c = 0; c < nv; ++c) {
    bound = fmax(bound, v[2 + c] + ax * v[10 + c]);
    if (nv == 4) bound = fmax(bound, v[6 + c] + ay * v[10 + c]);
  }
  const double limit = f32 ? 1e17 : 1e26;
  if (!(bound <= limit))
    return set_error(WZN_ERR_RANGE,
                     "split fluxes may reach %.3g, beyond the %.0e the weights are evaluated for",
                     bound, limit);
  return WZN_OK;
}

static const double RK_A[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
static const double RK_B[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};

int rk3_run_1d(const wzn_params* p, double* u, double* stage, int64_t n, double dx, double cfl,
               int32_t nsteps, const double* dt_in, const double* alpha_in, double* dt_out,
               double* alpha_out, Workspace* ws, hipStream_t s) {
  const int nv = p->system == WZN_EULER ? 3 : 1;
  const int64_t M = (int64_t)nv * n;
  double* U1 = stage;
  double* U2 = stage + M;
  const bool reduce_alpha = alpha_in == nullptr && p->lf_alpha_x < 0.0 && nv == 3;
  const bool cfl_dt = dt_in == nullptr;
  const bool need_speed = nv == 3 && (reduce_alpha || cfl_dt);
  const Tuning1D tn = tuning_1d(nv, n);
  unsigned long long* ring = ws->speed;
  int st = WZN_OK;
  if (need_speed) {
    st = launch_zero_words(ring, 3, s);
    if (st) return st;
    st = launch_speed_max<double>(u, n, 3, p->gamma, &ring[0], nullptr, s);
    if (st) return st;
  }
  if (nv == 1 && cfl_dt && nsteps > 0) {
    // advection: dt = cfl dx / |a|, a constant of the run
    st = launch_fill_double(ws->dt, cfl * dx / __builtin_fabs(p->adv_speed), s);
    if (st) return st;
  }
  const double const_alpha =
      p->lf_alpha_x >= 0.0 ? p->lf_alpha_x : __builtin_fabs(p->adv_speed);
  int64_t sidx = 0;
  for (int32_t step = 0; step < nsteps; ++step) {
    for (int k = 0; k < 3; ++k, ++sidx) {
      RowArgs<double> a = base_args(p, n, dx);
      a.mode = MODE_STAGE;
      a.uin = k == 0 ? u : (k == 1 ? U1 : U2);
      a.out = k == 0 ? U1 : (k == 1 ? U2 : u);
      a.un = k == 0 ? nullptr : u;
      a.rk_a = RK_A[k];
      a.rk_b = RK_B[k];
      unsigned long long* cur = &ring[sidx % 3];
      if (alpha_in) a.alpha_arr = alpha_in + 3 * step + k;
      else if (reduce_alpha) a.alpha_slot = cur;
      else a.alpha_const = const_alpha;
      if (dt_in) {
        a.dt_arr = dt_in + step;
      } else if (nv == 1) {
        a.dt_arr = ws->dt;
      } else if (k == 0) {
        a.dt_speed_slot = cur;
        a.cfl = cfl;
        a.dt_slot_write = ws->dt;
      } else {
        a.dt_slot_read = ws->dt;
      }
      if (dt_out && k == 0) a.dt_rec = dt_out + step;
      if (alpha_out) a.alpha_rec = alpha_out + 3 * step + k;
      if (need_speed) {
        // when alpha is frozen only U^{n+1} (k == 2) feeds a slot, for the next step's dt
        if (reduce_alpha || k == 2) a.speed_next = &ring[(sidx + 1) % 3];
        a.slot_zero = &ring[(sidx + 2) % 3];
      }
      st = launch_rows(a, sys_of(p), 1, tn, s);
      if (st) return st;
    }
  }
  return WZN_OK;
}

}  // namespace wzn
