// One row tile of the WENO-ZN hot path, shared by the row kernel (1D right-hand side / RK
// stage, 2D x sweep) and the persistent batched kernel.
//
// For a tile of T = NT*K consecutive cells of one row it evaluates
//   a1  boundary conditions as an index map in the tile loader (periodic wrap or
//       transmissive copy of the edge cell; Sec. 4.2, eq:26),
//   a2  the physical flux (advection a u; 1D Euler (rho u, rho u^2 + p, u (E + p)),
//       Sec. 4.3; 2D Euler x flux F of Sec. 4.4, eq:2d),
//   a3  the Lax-Friedrichs split w^{+-} = F +- alpha U (= 2 f^{+-}) with the global alpha,
//   a4  the WENO-ZN reconstruction of every interface (Sec. 3), fhat^- from the mirrored
//       window (Sec. 2),
//   a5  the conservative difference L = -(fhat_{i+1/2} - fhat_{i-1/2}) / dx (Sec. 2, eq:2),
//   a6  (stage mode) the TVD-RK3 stage combination out = a_s U^n + b_s (U + dt L) (Sec. 4),
//   and, on request, max(|u| + c) of the output cells (Sec. 4.3) into the caller's running max.
//
// Every interface flux is computed exactly once: thread t reconstructs the right interfaces
// of local cells tK .. tK+K-1 on a register sliding window, and the tile's left boundary
// interface (right interface of local cell -1) is computed by 2*NV lanes of wave 0, one
// (component, sign) reconstruction each.  Split fluxes are staged in LDS in a transposed
// layout (position p -> (p mod K) * LD + p / K) so that lane t reading position t*K + m hits
// consecutive words for every m.
#pragma once
#include <hip/hip_runtime.h>

#include "wzn_device.hpp"
#include "wzn_rows.hpp"

namespace wzn {

template <int SYS> struct SysInfo;
template <> struct SysInfo<SYS_ADV> { static constexpr int NV = 1; };
template <> struct SysInfo<SYS_EULER1> { static constexpr int NV = 3; };
template <> struct SysInfo<SYS_EULER2X> { static constexpr int NV = 4; };

// Physical flux along the row direction.
template <int SYS, typename T>
__device__ __forceinline__ void row_flux(const T* U, T* F, T adv, T gm1) {
  if constexpr (SYS == SYS_ADV) {
    F[0] = adv * U[0];
  } else if constexpr (SYS == SYS_EULER1) {
    const T rho = U[0], m = U[1], E = U[2];
    const T u = m / rho;
    const T p = gm1 * (E - (T(0.5) * rho) * u * u);
    F[0] = rho * u;
    F[1] = (rho * u) * u + p;
    F[2] = u * (E + p);
  } else {
    const T rho = U[0], mx = U[1], my = U[2], E = U[3];
    const T u = mx / rho, v = my / rho;
    const T p = gm1 * (E - (T(0.5) * rho) * (u * u + v * v));
    F[0] = mx;
    F[1] = mx * u + p;
    F[2] = mx * v;
    F[3] = u * (E + p);
  }
}

// Largest wave speed of a 1D state, evaluated without contraction so that every kernel that
// needs it (reductions, stage epilogues, the batched launch) gets the same bits.
template <int SYS>
__device__ __forceinline__ double wave_speed_1d(const double* U, double adv, double gamma) {
#pragma clang fp contract(off)
  if constexpr (SYS == SYS_ADV) {
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
  static constexpr int T = NT * K;      // cells (= right interfaces) per tile
  static constexpr int NP = T + 6;      // staged positions: local cells -3 .. T+2
  static constexpr int LD = (NP + K - 1) / K + 1;
  static constexpr int SZ = K * LD;     // elements per staged array
};

template <int NT, int K>
__device__ __forceinline__ int tpos(int p) {
  return (p % K) * Tile<NT, K>::LD + p / K;
}

template <int NT, int K, int SYS, typename T>
constexpr size_t tile_lds_bytes() {
  return sizeof(T) * (size_t)(2 * SysInfo<SYS>::NV) * Tile<NT, K>::SZ;
}

// Process the tile whose local cell 0 is global cell g0 of the row starting at element
// `rowoff` of every component plane.  W: dynamic LDS of tile_lds_bytes(); EX: 2*NV
// elements of LDS.  All threads of the workgroup must call it (it contains barriers).
template <int NT, int K, int SYS, typename T, bool SPEED>
__device__ __forceinline__ void row_tile(const RowArgs<T>& a, int64_t g0, int64_t rowoff,
                                         T alpha, double dt, T* W, T* EX, double& smax) {
  using TL = Tile<NT, K>;
  constexpr int TT = TL::T;
  constexpr int NV = SysInfo<SYS>::NV;
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  const T gm1 = T(a.gamma) - T(1);
  const T adv = T(a.adv);

  __syncthreads();  // the previous tile (if any) has finished reading LDS
  // ---- load: main rounds keep the cell state in registers for the epilogue
  T Ureg[K][NV];
#pragma unroll
  for (int r = 0; r <= K; ++r) {
    int p;
    if (r < K) p = 3 + tid + NT * r;                     // local cells 0 .. T-1
    else p = tid < 3 ? tid : (tid < 6 ? TT + tid : -1);  // cells -3,-2,-1, T,T+1,T+2
    if (r == K && p < 0) break;
    const int64_t gi = rowoff + bc_index(g0 + p - 3, n, a.bc);
    T U[NV], F[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) U[c] = a.uin[c * a.plane + gi];
    row_flux<SYS, T>(U, F, adv, gm1);
    const int q = tpos<NT, K>(p);
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      W[(2 * c + 0) * TL::SZ + q] = fma_t(alpha, U[c], F[c]);
      W[(2 * c + 1) * TL::SZ + q] = fma_t(-alpha, U[c], F[c]);
    }
    if (r < K) {
#pragma unroll
      for (int c = 0; c < NV; ++c) Ureg[r][c] = U[c];
    }
  }
  __syncthreads();

  const T eps_s = T(a.eps_s), A = T(a.A);
  // ---- left boundary interface of the tile: one (component, sign) per lane
  if (tid < 2 * NV) {
    const int c = tid >> 1, sg = tid & 1;
    T v[5], h[1];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const int p = sg == 0 ? i : 5 - i;  // w^+ at cells -3..1; w^- mirrored, cells 2..-2
      v[i] = W[(2 * c + sg) * TL::SZ + tpos<NT, K>(p)];
    }
    wzn_window<1>(v, h, eps_s, A);
    EX[tid] = h[0];
  }

  // ---- reconstruction: thread t owns the right interfaces of local cells tK .. tK+K-1
  T fh[NV][K];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    T v[K + 4], h[K];
    // w^+ at local cells tK-2 .. tK+K+1  (positions tK+1 .. tK+K+4)
#pragma unroll
    for (int i = 0; i < K + 4; ++i)
      v[i] = W[(2 * c) * TL::SZ + ((1 + i) % K) * TL::LD + tid + (1 + i) / K];
    wzn_window<K>(v, h, eps_s, A);
#pragma unroll
    for (int m = 0; m < K; ++m) fh[c][m] = h[m];
    // w^- mirrored: window r[i] = w^- at position tK + K + 5 - i (local cell tK + K + 2 - i)
#pragma unroll
    for (int i = 0; i < K + 4; ++i) {
      const int pp = K + 5 - i;
      v[i] = W[(2 * c + 1) * TL::SZ + (pp % K) * TL::LD + tid + pp / K];
    }
    wzn_window<K>(v, h, eps_s, A);
#pragma unroll
    for (int m = 0; m < K; ++m) fh[c][m] += h[K - 1 - m];
  }
  __syncthreads();  // all windows read; reuse LDS for the interface fluxes
  T* FH = W;        // [NV][SZ], indexed by local cell e in the transposed layout
#pragma unroll
  for (int c = 0; c < NV; ++c)
#pragma unroll
    for (int m = 0; m < K; ++m) FH[c * TL::SZ + m * TL::LD + tid] = fh[c][m];
  __syncthreads();

  // ---- epilogue on the loader mapping: local cell e = tid + NT r
  const T coef = T(-0.5 / a.dx);
#pragma unroll
  for (int r = 0; r < K; ++r) {
    const int e = tid + NT * r;
    const int64_t gcell = g0 + e;
    if (gcell >= n) continue;
    double O[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      const T fr = FH[c * TL::SZ + tpos<NT, K>(e)];
      const T fl = e > 0 ? FH[c * TL::SZ + tpos<NT, K>(e - 1)] : EX[2 * c] + EX[2 * c + 1];
      const T L = coef * (fr - fl);
      T o;
      if (a.mode == MODE_RHS) {
        o = L;
      } else {
        T v = Ureg[r][c] + T(dt) * L;
        if (a.un) v = fma_t(T(a.rk_a), a.un[c * a.plane + rowoff + gcell], T(a.rk_b) * v);
        o = v;
      }
      a.out[c * a.plane + rowoff + gcell] = o;
      O[c] = double(o);
    }
    if constexpr (SPEED && SYS != SYS_EULER2X) smax = fmax(smax, wave_speed_1d<SYS>(O, a.adv, a.gamma));
  }
}

// Largest wave speeds (|u| + c, |v| + c) of a 2D state, without contraction.
__device__ __forceinline__ void wave_speeds_2d(double rho, double mx, double my, double E,
                                               double gamma, double& sx, double& sy) {
#pragma clang fp contract(off)
  const double vx = mx / rho, vy = my / rho;
  const double p = (gamma - 1.0) * (E - (0.5 * rho) * (vx * vx + vy * vy));
  const double c = __builtin_sqrt(gamma * p / rho);
  sx = __builtin_fabs(vx) + c;
  sy = __builtin_fabs(vy) + c;
}

// Workgroup-wide max of per-thread values (all threads receive it).
template <int NT>
__device__ __forceinline__ double block_max(double v, double* red) {
  v = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = red[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) m = fmax(m, red[w]);
  return m;
}

}  // namespace wzn
