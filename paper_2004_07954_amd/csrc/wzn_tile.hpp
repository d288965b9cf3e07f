// One row tile of the WENO-ZN hot path, shared by the row kernel (1D right-hand side / RK
// stage, 2D x sweep) and the persistent batched kernel.
//
// For a tile of T = NT*K consecutive cells of one row it evaluates
//   a1  boundary conditions as an index map in the tile loader (periodic wrap or
//       transmissive copy of the edge cell; Sec. 4.2, eq:26),
//   a2  the physical flux (advection a u; 1D Euler (m, m u + p, u (E + p)),
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

// Velocity and pressure of a 1D Euler state: u = m / rho, p = (gamma - 1)(E - m u / 2)
// (Sec. 4.3), through one reciprocal of rho; fixed operation order so that every kernel that
// evaluates a flux gets the same bits.
template <typename T>
__device__ __forceinline__ void euler1_prim(T rho, T m, T E, T gm1, T& u, T& p) {
#pragma clang fp contract(off)
  u = m * rcp_nr(rho);
  p = gm1 * fma_t(-(T(0.5) * m), u, E);
}

// Component c of the 1D Euler flux (m, m u + p, u (E + p)).
template <typename T>
__device__ __forceinline__ T euler1_flux_comp(int c, T m, T E, T u, T p) {
#pragma clang fp contract(off)
  return c == 0 ? m : (c == 1 ? fma_t(m, u, p) : u * (E + p));
}

// Physical flux along the row direction.
template <int SYS, typename T>
__device__ __forceinline__ void row_flux(const T* U, T* F, T adv, T gm1) {
#pragma clang fp contract(off)
  if constexpr (SYS == SYS_ADV) {
    F[0] = adv * U[0];
  } else if constexpr (SYS == SYS_EULER1) {
    T u, p;
    euler1_prim<T>(U[0], U[1], U[2], gm1, u, p);
#pragma unroll
    for (int c = 0; c < 3; ++c) F[c] = euler1_flux_comp<T>(c, U[1], U[2], u, p);
  } else {
    const T rho = U[0], mx = U[1], my = U[2], E = U[3];
    const T r = rcp_nr(rho);
    const T u = mx * r, v = my * r;
    const T p = gm1 * fma_t(-(T(0.5) * my), v, fma_t(-(T(0.5) * mx), u, E));
    F[0] = mx;
    F[1] = fma_t(mx, u, p);
    F[2] = mx * v;
    F[3] = u * (E + p);
  }
}

// Largest wave speed |u| + c of a 1D state, c = sqrt(gamma p / rho), in a fixed operation
// order so that every kernel that needs it (reductions, stage epilogues, the batched launch)
// gets the same bits.
template <int SYS>
__device__ __forceinline__ double wave_speed_1d(const double* U, double adv, double gamma) {
#pragma clang fp contract(off)
  if constexpr (SYS == SYS_ADV) {
    return __builtin_fabs(adv);
  } else {
    const double r = rcp_nr(U[0]);
    const double u = U[1] * r;
    const double p = (gamma - 1.0) * (U[2] - (0.5 * U[1]) * u);
    return __builtin_fabs(u) + sqrt_gs((gamma * p) * r);
  }
}

// TVD-RK3 stage combination (Sec. 4) out = a_s U^n + b_s (U + dt L), evaluated as
// fma(b_s dt, L, base) with base = fma(a_s, U^n, b_s U) (base = U in the first stage, where
// a_s = 0, b_s = 1 and no U^n is read).  `ok` = false skips the U^n read (cells past the row).
template <typename T>
__device__ __forceinline__ T stage_base(const RowArgs<T>& a, T U, int64_t un_index, bool ok) {
  const T b = T(a.rk_b) * U;
  if (!a.un) return b;
  const T un = ok ? a.un[un_index] : T(0);
  return fma_t(T(a.rk_a), un, b);
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

// LDS of one tile: split fluxes of every component and both signs (SPLIT = false), or of one
// sign at a time (SPLIT = true: the two signs are staged and reconstructed one after the other,
// halving the footprint at the price of a second flux evaluation per cell).  The interface
// fluxes reuse the same space (NV arrays).
template <int NT, int K, int SYS, typename T, bool SPLIT = false>
constexpr size_t tile_lds_bytes() {
  return sizeof(T) * (size_t)((SPLIT ? 1 : 2) * SysInfo<SYS>::NV) * Tile<NT, K>::SZ;
}

// Process the tile whose local cell 0 is global cell g0 of the row starting at element
// `rowoff` of every component plane.  W: dynamic LDS of tile_lds_bytes(); EX: 2*NV
// elements of LDS.  All threads of the workgroup must call it (it contains barriers).
template <int NT, int K, int SYS, typename T, bool SPEED, bool SPLIT = false>
__device__ __forceinline__ void row_tile(const RowArgs<T>& a, int64_t g0, int64_t rowoff,
                                         T alpha, double dt, T* W, T* EX, double& smax) {
  using TL = Tile<NT, K>;
  constexpr int TT = TL::T;
  constexpr int NV = SysInfo<SYS>::NV;
  constexpr int NS = SPLIT ? 1 : 2;       // signs staged per phase
  constexpr int NPH = SPLIT ? 2 : 1;      // phases
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  const T gm1 = T(a.gamma) - T(1);
  const T adv = T(a.adv);
  const T eps_s = T(a.eps_s), A = window_const<T>(a.A);

  T Ureg[K][NV];
  T fh[NV][K];
#pragma unroll
  for (int ph = 0; ph < NPH; ++ph) {
    __syncthreads();  // LDS is free (previous tile or phase has finished reading it)
    // ---- load (first phase; main rounds keep the cell state in registers for the epilogue
    //      and the second phase), flux, split
#pragma unroll
    for (int r = 0; r <= K; ++r) {
      int p;
      if (r < K) p = 3 + tid + NT * r;                     // local cells 0 .. T-1
      else p = tid < 3 ? tid : (tid < 6 ? TT + tid : -1);  // cells -3,-2,-1, T,T+1,T+2
      if (r == K && p < 0) break;
      T U[NV], F[NV];
      if (ph == 0 || r == K) {
        const int64_t gi = rowoff + bc_index(g0 + p - 3, n, a.bc);
#pragma unroll
        for (int c = 0; c < NV; ++c) U[c] = a.uin[c * a.plane + gi];
      } else {
        // the second phase evaluates the flux again (not kept from the first phase, which
        // would hold NV*K more values across the whole reconstruction); the empty asm keeps
        // the compiler from reusing the first phase's results
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          U[c] = Ureg[r][c];
          asm volatile("" : "+v"(U[c]));
        }
      }
      row_flux<SYS, T>(U, F, adv, gm1);
      const int q = tpos<NT, K>(p);
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        if (!SPLIT || ph == 0) W[(NS * c) * TL::SZ + q] = fma_t(alpha, U[c], F[c]);
        if (!SPLIT || ph == 1) W[(NS * c + NS - 1) * TL::SZ + q] = fma_t(-alpha, U[c], F[c]);
      }
      if (ph == 0 && r < K) {
#pragma unroll
        for (int c = 0; c < NV; ++c) Ureg[r][c] = U[c];
      }
      if (SPLIT && ph == 1 && r < K && a.mode == MODE_STAGE) {
        // U is not needed past this point: replace it by the stage base a_s U^n + b_s U
        // (the U^n read is issued here, mid-kernel, rather than in the epilogue)
        const int64_t gcell = g0 + p - 3;
#pragma unroll
        for (int c = 0; c < NV; ++c)
          Ureg[r][c] = stage_base<T>(a, Ureg[r][c], c * a.plane + rowoff + gcell, gcell < n);
      }
    }
    __syncthreads();

    // ---- left boundary interface of the tile: one (component, sign) per lane
    if (tid < NS * NV) {
      const int c = tid / NS, sg = SPLIT ? ph : (tid & 1);
      T v[5], h[1];
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        const int p = sg == 0 ? i : 5 - i;  // w^+ at cells -3..1; w^- mirrored, cells 2..-2
        v[i] = W[(NS * c + (SPLIT ? 0 : sg)) * TL::SZ + tpos<NT, K>(p)];
      }
      wzn_window<1>(v, h, eps_s, A);
      EX[2 * c + sg] = h[0];
    }

    // ---- reconstruction: thread t owns the right interfaces of local cells tK .. tK+K-1
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      T v[K + 4], h[K];
      if (!SPLIT || ph == 0) {
        // w^+ at local cells tK-2 .. tK+K+1  (positions tK+1 .. tK+K+4)
#pragma unroll
        for (int i = 0; i < K + 4; ++i)
          v[i] = W[(NS * c) * TL::SZ + ((1 + i) % K) * TL::LD + tid + (1 + i) / K];
        wzn_window<K>(v, h, eps_s, A);
#pragma unroll
        for (int m = 0; m < K; ++m) {
          fh[c][m] = h[m];
          // materialise here: otherwise the compiler sinks the last steps of the window into
          // the second phase and keeps the window values alive across it
          if (SPLIT) asm volatile("" : "+v"(fh[c][m]));
        }
      }
      if (!SPLIT || ph == 1) {
        // w^- mirrored: r[i] = w^- at position tK + K + 5 - i (local cell tK + K + 2 - i)
#pragma unroll
        for (int i = 0; i < K + 4; ++i) {
          const int pp = K + 5 - i;
          v[i] = W[(NS * c + NS - 1) * TL::SZ + (pp % K) * TL::LD + tid + pp / K];
        }
        wzn_window<K>(v, h, eps_s, A);
#pragma unroll
        for (int m = 0; m < K; ++m) fh[c][m] += h[K - 1 - m];
      }
    }
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
        const T base = SPLIT ? Ureg[r][c]
                             : stage_base<T>(a, Ureg[r][c], c * a.plane + rowoff + gcell, true);
        o = fma_t(T(a.rk_b * dt), L, base);
      }
      a.out[c * a.plane + rowoff + gcell] = o;
      O[c] = double(o);
    }
    if constexpr (SPEED && SYS != SYS_EULER2X) smax = fmax(smax, wave_speed_1d<SYS>(O, a.adv, a.gamma));
  }
}

// Largest wave speeds (|u| + c, |v| + c) of a 2D state, in a fixed operation order.
__device__ __forceinline__ void wave_speeds_2d(double rho, double mx, double my, double E,
                                               double gamma, double& sx, double& sy) {
#pragma clang fp contract(off)
  const double r = rcp_nr(rho);
  const double vx = mx * r, vy = my * r;
  const double p = (gamma - 1.0) * ((E - (0.5 * mx) * vx) - (0.5 * my) * vy);
  const double c = sqrt_gs((gamma * p) * r);
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
