// 2D dimension-by-dimension WENO-ZN (Sec. 4.4, eq:2d) for gfx950, fp64 and fp32.
//
// One right-hand side is two kernels:
//   1. the row kernel (wzn_rows.hip) sweeps x: Lx = -(Fhat_{i+1/2,j} - Fhat_{i-1/2,j}) / dx,
//      with the Lax-Friedrichs split of F by alpha_x, written to a scratch plane set;
//   2. the column kernel below sweeps y and finishes the cell: L = Lx - (Ghat_{i,j+1/2} -
//      Ghat_{i,j-1/2}) / dy with the split of G by alpha_y, then the TVD-RK3 stage
//      combination, and max(|u| + c), max(|v| + c) of the output for the next stage's alphas
//      and the next step's dt = cfl dtx dty / (dtx + dty) (Sec. 4.4).
//
// Column kernel layout: a wave covers 64 consecutive columns (lane = column, so every global
// access of a row is coalesced); each lane walks down one column segment of S = KY*R - 1
// rows in R chunks of KY interfaces.  The chunk window (KY + 5 rows) lives in registers
// together with the primitive state of each row (rho, rho u, rho v, E, v, p), and the five
// rows shared with the next chunk are carried over instead of reloaded.  The segment's
// first interface (below its first row) is the one extra interface per segment.
#include <hip/hip_runtime.h>

#include "wzn_device.hpp"
#include "wzn_host.hpp"
#include "wzn_rows.hpp"
#include "wzn_tile.hpp"

namespace wzn {

template <typename T>
struct ColArgs {
  const T* uin;   // stage input [4][ny][nx]
  const T* lx;    // x part of L from the row kernel, [4][ny][nx]
  const T* un;    // U^n or null
  T* out;         // L (MODE_RHS) or U^(s+1); may alias lx (each element is read, then written,
                  // by the same thread)
  int64_t nx, ny, plane;
  double dx, dy;
  int bc;
  int mode;
  int nseg;       // segments along y
  double rk_a, rk_b;
  double gamma, eps_s, A;
  const unsigned long long* alpha_slot;  // alpha_y
  const double* alpha_arr;
  double alpha_const;
  const double* dt_arr;
  const unsigned long long* dt_speed_x;
  const unsigned long long* dt_speed_y;
  const double* dt_slot_read;
  double cfl;
  double* dt_slot_write;
  double* dt_rec;
  unsigned long long* speed_next_x;
  unsigned long long* speed_next_y;
  unsigned long long* zero_x;
  unsigned long long* zero_y;
};

template <typename T>
struct Prim {
  T rho, mx, my, E, v, p;
};

template <int KY, int R, int NW, typename T>
__global__ __launch_bounds__(64 * NW)
void col_kernel(ColArgs<T> a) {
  constexpr int S = KY * R - 1;  // rows per segment
  constexpr int NPOS = KY + 5;
  __shared__ double red[2][NW];
  const int lane = threadIdx.x;
  const int64_t x = (int64_t)blockIdx.x * 64 + lane;
  const int64_t xc = x < a.nx ? x : a.nx - 1;
  const int seg = blockIdx.y * NW + threadIdx.y;
  const int64_t r0 = (int64_t)seg * S;

  double alpha_d;
  if (a.alpha_slot) alpha_d = slot_value(a.alpha_slot);
  else if (a.alpha_arr) alpha_d = a.alpha_arr[0];
  else alpha_d = a.alpha_const;
  const T alpha = T(alpha_d);
  double dt = 0.0;
  if (a.mode == MODE_STAGE) {
    if (a.dt_arr) {
      dt = a.dt_arr[0];
    } else if (a.dt_speed_x) {
      const double dtx = a.dx / slot_value(a.dt_speed_x);
      const double dty = a.dy / slot_value(a.dt_speed_y);
      dt = a.cfl * dtx * dty / (dtx + dty);
    } else {
      dt = a.dt_slot_read[0];
    }
  }
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && threadIdx.y == 0) {
    if (a.dt_slot_write) a.dt_slot_write[0] = dt;
    if (a.dt_rec) a.dt_rec[0] = dt;
    if (a.zero_x) a.zero_x[0] = 0ull;
    if (a.zero_y) a.zero_y[0] = 0ull;
  }

  const T gm1 = T(a.gamma) - T(1);
  const T eps_s = T(a.eps_s), A = window_const<T>(a.A);
  const T coef = T(-0.5 / a.dy);
  const double gamma = a.gamma;
  double sxm = 0.0, sym = 0.0;

  if (seg < a.nseg) {
    Prim<T> P[NPOS];
    T carry[4];
    for (int ch = 0; ch < R; ++ch) {
      const int64_t q0 = r0 - 1 + (int64_t)ch * KY;  // first interface row of the chunk
#pragma unroll
      for (int i = 0; i < NPOS; ++i) {
        if (ch > 0 && i < 5) continue;  // carried over from the previous chunk
        const int64_t gy = bc_index(q0 - 2 + i, a.ny, a.bc);
        const int64_t gi = gy * a.nx + xc;
        Prim<T> q;
        q.rho = a.uin[gi];
        q.mx = a.uin[a.plane + gi];
        q.my = a.uin[2 * a.plane + gi];
        q.E = a.uin[3 * a.plane + gi];
        const T r = rcp_nr(q.rho);
        const T u = q.mx * r;
        q.v = q.my * r;
        q.p = gm1 * fma_t(-(T(0.5) * q.my), q.v, fma_t(-(T(0.5) * q.mx), u, q.E));
        P[i] = q;
      }
      // per component: reconstruct the KY top interfaces, then finish the KY rows
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        T G[NPOS], Uc[NPOS];
#pragma unroll
        for (int i = 0; i < NPOS; ++i) {
          const Prim<T>& q = P[i];
          if (c == 0) { G[i] = q.my; Uc[i] = q.rho; }
          else if (c == 1) { G[i] = q.mx * q.v; Uc[i] = q.mx; }
          else if (c == 2) { G[i] = fma_t(q.my, q.v, q.p); Uc[i] = q.my; }
          else { G[i] = q.v * (q.E + q.p); Uc[i] = q.E; }
        }
        T w[KY + 4], h[KY], fh[KY];
#pragma unroll
        for (int i = 0; i < KY + 4; ++i) w[i] = fma_t(alpha, Uc[i], G[i]);
        wzn_window<KY>(w, h, eps_s, A);
#pragma unroll
        for (int m = 0; m < KY; ++m) fh[m] = h[m];
#pragma unroll
        for (int i = 0; i < KY + 4; ++i) w[i] = fma_t(-alpha, Uc[KY + 4 - i], G[KY + 4 - i]);
        wzn_window<KY>(w, h, eps_s, A);
#pragma unroll
        for (int m = 0; m < KY; ++m) fh[m] += h[KY - 1 - m];
        // rows q0 + m: bottom interface fh[m-1] (or the one carried from the last chunk)
#pragma unroll
        for (int m = 0; m < KY; ++m) {
          const int64_t y = q0 + m;
          const bool active = (ch > 0 || m > 0) && y < r0 + S && y < a.ny && x < a.nx;
          if (active) {
            const int64_t gi = y * a.nx + x;
            const T lo = m > 0 ? fh[m - 1] : carry[c];
            const T L = a.lx[c * a.plane + gi] + coef * (fh[m] - lo);
            T o;
            if (a.mode == MODE_RHS) {
              o = L;
            } else {
              T v = Uc[m + 2] + T(dt) * L;
              if (a.un) v = fma_t(T(a.rk_a), a.un[c * a.plane + gi], T(a.rk_b) * v);
              o = v;
            }
            a.out[c * a.plane + gi] = o;
          }
        }
        carry[c] = fh[KY - 1];
      }
      if (a.speed_next_x) {
#pragma unroll
        for (int m = 0; m < KY; ++m) {
          const int64_t y = q0 + m;
          const bool active = (ch > 0 || m > 0) && y < r0 + S && y < a.ny && x < a.nx;
          if (active) {
            // the thread re-reads the four components it has just written
            const int64_t gi = y * a.nx + x;
            const double o0 = a.out[gi], o1 = a.out[a.plane + gi];
            const double o2 = a.out[2 * a.plane + gi], o3 = a.out[3 * a.plane + gi];
            double ax, ay;
            wave_speeds_2d(o0, o1, o2, o3, gamma, ax, ay);
            sxm = fmax(sxm, ax);
            sym = fmax(sym, ay);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 5; ++i) P[i] = P[i + KY];
    }
  }
  if (a.speed_next_x) {
    sxm = wave_max(sxm);
    sym = wave_max(sym);
    if (lane == 0) {
      red[0][threadIdx.y] = sxm;
      red[1][threadIdx.y] = sym;
    }
    __syncthreads();
    if (lane == 0 && threadIdx.y == 0) {
      double mx = red[0][0], my = red[1][0];
#pragma unroll
      for (int w = 1; w < NW; ++w) {
        mx = fmax(mx, red[0][w]);
        my = fmax(my, red[1][w]);
      }
      atomic_max_pos(a.speed_next_x, mx);
      atomic_max_pos(a.speed_next_y, my);
    }
  }
}

template <int KY, int R, int NW, typename T>
static int launch_col_t(ColArgs<T> a, hipStream_t s) {
  constexpr int S = KY * R - 1;
  a.nseg = (int)((a.ny + S - 1) / S);
  const int64_t bx = (a.nx + 63) / 64;
  const int64_t by = (a.nseg + NW - 1) / NW;
  if (bx > 0x7fffffff || by > 65535) return set_error(WZN_ERR_SIZE, "grid too large (columns)");
  hipLaunchKernelGGL((col_kernel<KY, R, NW, T>), dim3((unsigned)bx, (unsigned)by), dim3(64, NW), 0,
                     s, a);
  return check_launch("col_kernel");
}

// ------------------------------------------------------------------ host side
template <typename T>
static RowArgs<T> row_args(const wzn_params* p, int64_t nx, int64_t ny, double dx) {
  RowArgs<T> a{};
  a.n = nx;
  a.plane = nx * ny;
  a.row_stride = nx;
  a.dx = dx;
  a.bc = p->bc_x;
  a.mode = MODE_RHS;
  a.gamma = p->gamma;
  a.eps_s = 16.0 * p->eps;
  a.A = p->A;
  return a;
}

template <typename T>
static ColArgs<T> col_args(const wzn_params* p, int64_t nx, int64_t ny, double dx, double dy) {
  ColArgs<T> a{};
  a.nx = nx;
  a.ny = ny;
  a.plane = nx * ny;
  a.dx = dx;
  a.dy = dy;
  a.bc = p->bc_y;
  a.gamma = p->gamma;
  a.eps_s = 16.0 * p->eps;
  a.A = p->A;
  return a;
}

static Tuning1D tuning_2dx() { return Tuning1D{256, 4, ROW_LDS_TILE}; }

template <typename T>
int rhs_2d_t(const wzn_params* p, const T* u, T* dudt, int64_t nx, int64_t ny, double dx,
             double dy, Workspace* ws, hipStream_t s) {
  RowArgs<T> ra = row_args<T>(p, nx, ny, dx);
  ColArgs<T> ca = col_args<T>(p, nx, ny, dx, dy);
  const bool reduce = p->lf_alpha_x < 0.0 || p->lf_alpha_y < 0.0;
  if (reduce) {
    int st = launch_zero_words(ws->speed, 6, s);
    if (st) return st;
    st = launch_speed_max<T>(u, nx * ny, 4, p->gamma, &ws->speed[0], &ws->speed_y[0], s);
    if (st) return st;
  }
  if (p->lf_alpha_x >= 0.0) ra.alpha_const = p->lf_alpha_x;
  else ra.alpha_slot = &ws->speed[0];
  if (p->lf_alpha_y >= 0.0) ca.alpha_const = p->lf_alpha_y;
  else ca.alpha_slot = &ws->speed_y[0];
  ra.uin = u;
  ra.out = dudt;
  int st = launch_rows(ra, SYS_EULER2X, ny, tuning_2dx(), s);
  if (st) return st;
  ca.uin = u;
  ca.lx = dudt;
  ca.out = dudt;
  ca.mode = MODE_RHS;
  return launch_col_t<4, 16, 4, T>(ca, s);
}
template int rhs_2d_t<double>(const wzn_params*, const double*, double*, int64_t, int64_t, double,
                              double, Workspace*, hipStream_t);
template int rhs_2d_t<float>(const wzn_params*, const float*, float*, int64_t, int64_t, double,
                             double, Workspace*, hipStream_t);

static const double RK_A[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
static const double RK_B[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};

template <typename T>
int rk3_run_2d_t(const wzn_params* p, T* u, T* stage, int64_t nx, int64_t ny, double dx,
                 double dy, double cfl, int32_t nsteps, const double* dt_in, double* dt_out,
                 Workspace* ws, hipStream_t s) {
  const int64_t M = 4 * nx * ny;
  T* U1 = stage;
  T* U2 = stage + M;
  const bool reduce_x = p->lf_alpha_x < 0.0, reduce_y = p->lf_alpha_y < 0.0;
  const bool need_speed = reduce_x || reduce_y || dt_in == nullptr;
  unsigned long long* rx = ws->speed;
  unsigned long long* ry = ws->speed_y;
  int st;
  if (need_speed) {
    st = launch_zero_words(ws->speed, 6, s);
    if (st) return st;
    st = launch_speed_max<T>(u, nx * ny, 4, p->gamma, &rx[0], &ry[0], s);
    if (st) return st;
  }
  int64_t sidx = 0;
  for (int32_t step = 0; step < nsteps; ++step) {
    for (int k = 0; k < 3; ++k, ++sidx) {
      const T* in = k == 0 ? u : (k == 1 ? U1 : U2);
      T* out = k == 0 ? U1 : (k == 1 ? U2 : u);
      T* scratch = k == 1 ? U2 : U1;  // holds Lx; never the stage input or U^n
      const int cur = (int)(sidx % 3), nxt = (int)((sidx + 1) % 3), old = (int)((sidx + 2) % 3);
      RowArgs<T> ra = row_args<T>(p, nx, ny, dx);
      ra.uin = in;
      ra.out = scratch;
      if (reduce_x) ra.alpha_slot = &rx[cur];
      else ra.alpha_const = p->lf_alpha_x;
      st = launch_rows(ra, SYS_EULER2X, ny, tuning_2dx(), s);
      if (st) return st;
      ColArgs<T> ca = col_args<T>(p, nx, ny, dx, dy);
      ca.uin = in;
      ca.lx = scratch;
      ca.out = out;
      ca.un = k == 0 ? nullptr : u;
      ca.mode = MODE_STAGE;
      ca.rk_a = RK_A[k];
      ca.rk_b = RK_B[k];
      if (reduce_y) ca.alpha_slot = &ry[cur];
      else ca.alpha_const = p->lf_alpha_y;
      if (dt_in) {
        ca.dt_arr = dt_in + step;
      } else if (k == 0) {
        ca.dt_speed_x = &rx[cur];
        ca.dt_speed_y = &ry[cur];
        ca.cfl = cfl;
        ca.dt_slot_write = ws->dt;
      } else {
        ca.dt_slot_read = ws->dt;
      }
      if (dt_out && k == 0) ca.dt_rec = dt_out + step;
      if (need_speed) {
        if (reduce_x || reduce_y || k == 2) {
          ca.speed_next_x = &rx[nxt];
          ca.speed_next_y = &ry[nxt];
        }
        ca.zero_x = &rx[old];
        ca.zero_y = &ry[old];
      }
      st = launch_col_t<4, 16, 4, T>(ca, s);
      if (st) return st;
    }
  }
  return WZN_OK;
}
template int rk3_run_2d_t<double>(const wzn_params*, double*, double*, int64_t, int64_t, double,
                                  double, double, int32_t, const double*, double*, Workspace*,
                                  hipStream_t);
template int rk3_run_2d_t<float>(const wzn_params*, float*, float*, int64_t, int64_t, double,
                                 double, double, int32_t, const double*, double*, Workspace*,
                                 hipStream_t);

}  // namespace wzn
