// 1D WENO-ZN right-hand side and fused TVD-RK3 stages for gfx950, fp64.
//
// One kernel evaluates, per workgroup tile of T = NT*K interfaces:
//   a1  boundary conditions as an index map in the tile loader (periodic wrap or
//       transmissive copy; Sec. 4.2, eq:26),
//   a2  the physical flux (advection a u; Euler (rho u, rho u^2 + p, u (E + p)), Sec. 4.3),
//   a3  the Lax-Friedrichs split w^{+-} = F +- alpha U (= 2 f^{+-}) with the global alpha,
//   a4  the WENO-ZN reconstruction of every interface (Sec. 3) -- fhat^- from the mirrored
//       window (Sec. 2),
//   a5  the conservative difference L = -(fhat_{i+1/2} - fhat_{i-1/2}) / dx (Sec. 2, eq:2),
//   a6  the TVD-RK3 stage combination out = a_s U^n + b_s (U + dt L) (Sec. 4),
//   and, in the epilogue, max(|u| + c) of the stage output for the next stage's alpha and the
//   next step's dt (Sec. 4.3), folded into one atomic per workgroup.
//
// Tiles overlap by one cell: a tile computes the T right-interface fluxes of its local cells
// 0..T-1 and updates cells 1..T-1, so every interface flux of the tile is computed exactly
// once and no thread does extra work.  Split fluxes are staged in LDS in a transposed layout
// (position p -> (p mod K) * LD + p / K) so that lane t reading position t*K + m hits
// consecutive words for every m.
#include <hip/hip_runtime.h>

#include "wzn_device.hpp"
#include "wzn_host.hpp"

namespace wzn {

enum { MODE_RHS = 0, MODE_STAGE = 1 };

struct Stage1DArgs {
  const double* uin;  // stage input U^(s)  [nv][n]
  const double* un;   // U^n (stage combination) or null when a_s == 0
  double* out;        // L (MODE_RHS) or U^(s+1) (MODE_STAGE)
  int64_t n;
  double dx;
  int bc;
  int mode;
  double rk_a, rk_b;
  double adv, gamma, eps_s, A;
  // LF alpha of this RHS evaluation: slot (reduced) / array (frozen) / constant
  const unsigned long long* alpha_slot;
  const double* alpha_arr;
  double alpha_const;
  // dt: array / from the alpha of U^n in a slot / from the dt slot
  const double* dt_arr;
  const unsigned long long* dt_speed_slot;
  const double* dt_slot_read;
  double cfl;
  double* dt_slot_write;
  double* dt_rec;
  double* alpha_rec;
  // epilogue
  unsigned long long* speed_next;  // atomic max of |u| + c of the output, or null
  unsigned long long* slot_zero;   // zeroed by workgroup 0, or null
};

template <int NV>
__device__ __forceinline__ void phys_flux(const double* U, double* F, double adv, double gm1) {
  if constexpr (NV == 1) {
    F[0] = adv * U[0];
  } else {
    const double rho = U[0], m = U[1], E = U[2];
    const double u = m / rho;
    const double p = gm1 * (E - (0.5 * rho) * u * u);
    F[0] = rho * u;
    F[1] = (rho * u) * u + p;
    F[2] = u * (E + p);
  }
}

template <int NV>
__device__ __forceinline__ double wave_speed(const double* U, double adv, double gamma) {
  if constexpr (NV == 1) {
    return __builtin_fabs(adv);
  } else {
    const double rho = U[0], m = U[1], E = U[2];
    const double u = m / rho;
    const double p = (gamma - 1.0) * (E - (0.5 * rho) * u * u);
    return __builtin_fabs(u) + __builtin_sqrt(gamma * p / rho);
  }
}

template <int NT, int K>
struct Tile {
  static constexpr int T = NT * K;      // interfaces per tile
  static constexpr int NP = T + 5;      // staged positions (local cells -2 .. T+2)
  static constexpr int LD = (NP + K - 1) / K + 1;
  static constexpr int SZ = K * LD;     // doubles per staged array
};

template <int NT, int K>
__device__ __forceinline__ int tpos(int p) {
  return (p % K) * Tile<NT, K>::LD + p / K;
}

template <int NT, int K, int NV>
__global__ __launch_bounds__(NT) void stage1d_kernel(Stage1DArgs a) {
  using TL = Tile<NT, K>;
  constexpr int T = TL::T;
  extern __shared__ double lds[];
  double* W = lds;  // [NV][2][SZ]: w^+ then w^- per component

  const int tid = threadIdx.x;
  const int64_t n = a.n;
  const int64_t g0 = (int64_t)blockIdx.x * (T - 1) - 1;  // global index of local cell 0

  // ---- alpha and dt of this evaluation (uniform per kernel)
  double alpha;
  if (a.alpha_slot) alpha = slot_value(a.alpha_slot);
  else if (a.alpha_arr) alpha = a.alpha_arr[0];
  else alpha = a.alpha_const;
  double dt = 0.0;
  if (a.mode == MODE_STAGE) {
    if (a.dt_arr) dt = a.dt_arr[0];
    else if (a.dt_speed_slot) dt = a.cfl * a.dx / slot_value(a.dt_speed_slot);
    else dt = a.dt_slot_read[0];
  }
  if (blockIdx.x == 0 && tid == 0) {
    if (a.dt_slot_write) a.dt_slot_write[0] = dt;
    if (a.dt_rec) a.dt_rec[0] = dt;
    if (a.alpha_rec) a.alpha_rec[0] = alpha;
    if (a.slot_zero) a.slot_zero[0] = 0ull;
  }

  const double gm1 = a.gamma - 1.0;
  // ---- load: main rounds keep the cell state in registers for the epilogue
  double Ureg[K][NV];
#pragma unroll
  for (int r = 0; r <= K; ++r) {
    int p;
    if (r < K) p = 3 + tid + NT * r;                       // local cells 1 .. T
    else p = tid < 3 ? tid : (tid < 5 ? T + tid - 3 + 3 : -1);  // cells -2,-1,0,T+1,T+2
    if (r == K && p < 0) break;
    const int64_t gi = bc_index(g0 + p - 2, n, a.bc);
    double U[NV], F[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) U[c] = a.uin[c * n + gi];
    phys_flux<NV>(U, F, a.adv, gm1);
    const int q = tpos<NT, K>(p);
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      W[(2 * c + 0) * TL::SZ + q] = __builtin_fma(alpha, U[c], F[c]);
      W[(2 * c + 1) * TL::SZ + q] = __builtin_fma(-alpha, U[c], F[c]);
    }
    if (r < K) {
#pragma unroll
      for (int c = 0; c < NV; ++c) Ureg[r][c] = U[c];
    }
  }
  __syncthreads();

  // ---- reconstruction: thread t owns the right interfaces of local cells tK .. tK+K-1
  double fh[NV][K];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    double v[K + 4], h[K];
    // w^+ at local cells tK-2 .. tK+K+1  (positions tK .. tK+K+3)
#pragma unroll
    for (int i = 0; i < K + 4; ++i) v[i] = W[(2 * c) * TL::SZ + (i % K) * TL::LD + tid + i / K];
    wzn_window<K>(v, h, a.eps_s, a.A);
#pragma unroll
    for (int m = 0; m < K; ++m) fh[c][m] = h[m];
    // w^- mirrored: window r[i] = w^- at position tK + K + 4 - i  (i = 0 .. K+3)
#pragma unroll
    for (int i = 0; i < K + 4; ++i) {
      const int pp = K + 4 - i;  // position offset from tK
      v[i] = W[(2 * c + 1) * TL::SZ + (pp % K) * TL::LD + tid + pp / K];
    }
    wzn_window<K>(v, h, a.eps_s, a.A);
#pragma unroll
    for (int m = 0; m < K; ++m) fh[c][m] += h[K - 1 - m];
  }
  __syncthreads();  // all windows read; reuse LDS for the interface fluxes
  double* FH = lds;  // [NV][SZ], indexed by local cell e in the transposed layout
#pragma unroll
  for (int c = 0; c < NV; ++c)
#pragma unroll
    for (int m = 0; m < K; ++m) FH[c * TL::SZ + m * TL::LD + tid] = fh[c][m];
  __syncthreads();

  // ---- epilogue on the loader mapping: local cell e = 1 + tid + NT r
  const double coef = -0.5 / a.dx;
  double smax = 0.0;
#pragma unroll
  for (int r = 0; r < K; ++r) {
    const int e = 1 + tid + NT * r;
    const int64_t gcell = g0 + e;
    if (e > T - 1 || gcell >= n) continue;
    double O[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      const double fr = FH[c * TL::SZ + tpos<NT, K>(e)];
      const double fl = FH[c * TL::SZ + tpos<NT, K>(e - 1)];
      const double L = coef * (fr - fl);
      if (a.mode == MODE_RHS) {
        O[c] = L;
      } else {
        double v = Ureg[r][c] + dt * L;
        if (a.un) v = __builtin_fma(a.rk_a, a.un[c * n + gcell], a.rk_b * v);
        O[c] = v;
      }
      a.out[c * n + gcell] = O[c];
    }
    if (a.speed_next) smax = fmax(smax, wave_speed<NV>(O, a.adv, a.gamma));
  }
  if (a.speed_next) {
    __shared__ double red[NT / 64];
    smax = wave_max(smax);
    if ((tid & 63) == 0) red[tid >> 6] = smax;
    __syncthreads();
    if (tid == 0) {
      double mm = red[0];
#pragma unroll
      for (int w = 1; w < NT / 64; ++w) mm = fmax(mm, red[w]);
      atomic_max_pos(a.speed_next, mm);
    }
  }
}

// max over cells of |u| + c into *slot (slot must be zero beforehand)
template <int NV>
__global__ __launch_bounds__(256) void speed_max_kernel(const double* __restrict__ u, int64_t n,
                                                        double adv, double gamma,
                                                        unsigned long long* slot) {
  double smax = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    double U[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) U[c] = u[c * n + i];
    smax = fmax(smax, wave_speed<NV>(U, adv, gamma));
  }
  __shared__ double red[4];
  smax = wave_max(smax);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = smax;
  __syncthreads();
  if (threadIdx.x == 0) atomic_max_pos(slot, fmax(fmax(red[0], red[1]), fmax(red[2], red[3])));
}

__global__ void zero_words_kernel(unsigned long long* p, int count) {
  const int i = threadIdx.x;
  if (i < count) p[i] = 0ull;
}

// ------------------------------------------------------------------ host side
template <int NT, int K>
static size_t stage_lds_bytes(int nv) {
  return sizeof(double) * (size_t)(2 * nv) * Tile<NT, K>::SZ;
}

template <int NT, int K, int NV>
static int launch_stage_t(const Stage1DArgs& a, hipStream_t s) {
  constexpr int T = NT * K;
  const int64_t blocks = (a.n + (T - 1) - 1) / (T - 1);
  const size_t lds = stage_lds_bytes<NT, K>(NV);
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute((const void*)stage1d_kernel<NT, K, NV>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return set_error(WZN_ERR_HIP, "hipFuncSetAttribute(stage1d_kernel) failed");
    attr_set = true;
  }
  hipLaunchKernelGGL((stage1d_kernel<NT, K, NV>), dim3((unsigned)blocks), dim3(NT), lds, s, a);
  return check_launch("stage1d_kernel");
}

static int launch_stage(const Stage1DArgs& a, int nv, const Tuning1D& tn, hipStream_t s) {
  // the autotuned configurations available in this build
  if (nv == 3) {
    if (tn.nt == 256 && tn.k == 4) return launch_stage_t<256, 4, 3>(a, s);
    if (tn.nt == 256 && tn.k == 2) return launch_stage_t<256, 2, 3>(a, s);
    if (tn.nt == 128 && tn.k == 4) return launch_stage_t<128, 4, 3>(a, s);
    if (tn.nt == 256 && tn.k == 1) return launch_stage_t<256, 1, 3>(a, s);
    if (tn.nt == 128 && tn.k == 8) return launch_stage_t<128, 8, 3>(a, s);
    if (tn.nt == 64 && tn.k == 8) return launch_stage_t<64, 8, 3>(a, s);
    return set_error(WZN_ERR_ARG, "unsupported 1D tuning (nt=%d, k=%d)", tn.nt, tn.k);
  }
  if (tn.nt == 256 && tn.k == 4) return launch_stage_t<256, 4, 1>(a, s);
  return launch_stage_t<64, 4, 1>(a, s);
}

static int launch_speed_max(const double* u, int64_t n, int nv, double adv, double gamma,
                            unsigned long long* slot, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (nv == 3)
    hipLaunchKernelGGL((speed_max_kernel<3>), dim3((unsigned)blocks), dim3(256), 0, s, u, n, adv,
                       gamma, slot);
  else
    hipLaunchKernelGGL((speed_max_kernel<1>), dim3((unsigned)blocks), dim3(256), 0, s, u, n, adv,
                       gamma, slot);
  return check_launch("speed_max_kernel");
}

int launch_zero_words(unsigned long long* p, int count, hipStream_t s) {
  hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, p, count);
  return check_launch("zero_words_kernel");
}

static Stage1DArgs base_args(const wzn_params* p, int64_t n, double dx) {
  Stage1DArgs a{};
  a.n = n;
  a.dx = dx;
  a.bc = p->bc_x;
  a.adv = p->adv_speed;
  a.gamma = p->gamma;
  a.eps_s = 16.0 * p->eps;
  a.A = p->A;
  return a;
}

int rhs_1d(const wzn_params* p, const double* u, double* dudt, int64_t n, double dx, Workspace* ws,
           hipStream_t s) {
  const int nv = p->system == WZN_EULER ? 3 : 1;
  Stage1DArgs a = base_args(p, n, dx);
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
    st = launch_speed_max(u, n, nv, p->adv_speed, p->gamma, ws->speed, s);
    if (st) return st;
    a.alpha_slot = ws->speed;
  }
  return launch_stage(a, nv, tuning_1d(nv, n), s);
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
  unsigned long long* ring = ws->speed;  // 3 slots
  int st = WZN_OK;
  if (need_speed) {
    st = launch_zero_words(ring, 3, s);
    if (st) return st;
    st = launch_speed_max(u, n, nv, p->adv_speed, p->gamma, &ring[0], s);
    if (st) return st;
  }
  const double const_alpha =
      p->lf_alpha_x >= 0.0 ? p->lf_alpha_x : __builtin_fabs(p->adv_speed);
  const double const_dt = nv == 1 ? cfl * dx / __builtin_fabs(p->adv_speed) : 0.0;
  int64_t sidx = 0;  // global stage counter for the slot ring
  for (int32_t step = 0; step < nsteps; ++step) {
    for (int k = 0; k < 3; ++k, ++sidx) {
      Stage1DArgs a = base_args(p, n, dx);
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
        a.dt_arr = ws->dt;  // cfl dx / |a|, filled once below
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
        // the next stage reads slot (sidx+1) % 3, which this kernel fills; the slot it zeroes
        // was last read by the previous kernel.  When alpha is not reduced only the stage-3
        // output (U^{n+1}) feeds a slot (for the next step's dt).
        if (reduce_alpha || k == 2) a.speed_next = &ring[(sidx + 1) % 3];
        a.slot_zero = &ring[(sidx + 2) % 3];
      }
      if (nv == 1 && !dt_in && step == 0 && k == 0) {
        st = launch_fill_double(ws->dt, const_dt, s);
        if (st) return st;
      }
      st = launch_stage(a, nv, tn, s);
      if (st) return st;
    }
  }
  return WZN_OK;
}

}  // namespace wzn
