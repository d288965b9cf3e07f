// Wave tile of the WENO-ZN hot path: one 64-lane wave evaluates a run of 64*K consecutive
// cells of one row with no LDS staging and no workgroup barrier.
//
// It computes what the LDS row tile (wzn_tile.hpp) computes, with the same arithmetic in the
// same order, so results are bit for bit those of the row tile:
//   a1  boundary conditions as an index map in the loader (periodic wrap or transmissive copy
//       of the edge cell; Sec. 4.2, eq:26),
//   a2  the physical flux (advection a u; 1D Euler, Sec. 4.3),
//   a3  the Lax-Friedrichs split w^{+-} = F +- alpha U (= 2 f^{+-}),
//   a4  the WENO-ZN reconstruction of every interface (Sec. 3), f^- from the mirrored window,
//   a5  the conservative difference L = -(fhat_{i+1/2} - fhat_{i-1/2}) / dx (Sec. 2, eq:2),
//   a6  (stage mode) the TVD-RK3 stage combination, and on request the max of |u| + c of the
//       output cells.
//
// Layout: lane l owns the K consecutive cells lK .. lK+K-1 of the run (contiguous loads and
// stores per lane), plus one halo cell on lanes 0..5 (run cells -3, -2, -1, 64K, 64K+1,
// 64K+2).  The sliding windows of a lane need two cells of w^+ to its left and right and one
// cell of w^- to the left and three to the right: they come from the neighbouring lanes by
// cross-lane permutes (ds_bpermute), and from the halo lanes by readlane at the two ends of
// the run.  The run's left boundary interface (right interface of run cell -1) is
// reconstructed once per component by lanes 0 (w^+) and 1 (mirrored w^-).  Each interface
// flux is computed exactly once; the left flux of lane l's first cell is lane l-1's last.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wzn_device.hpp"
#include "wzn_rows.hpp"
#include "wzn_tile.hpp"

namespace wzn {

__device__ __forceinline__ double readlane_t(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ float readlane_t(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// Value at run cell lane*K + D (D in [-2, 2K-1]) of a per-lane array w[K] of the wave, with
// the halo register h (lane 3 + t holds run cell t for t in [-3, -1], lane 3 + t - 64K holds
// run cell t for t in [64K, 64K+2]).  D is a compile-time constant after unrolling.
template <int K, typename T>
__device__ __forceinline__ T run_cell(const T (&w)[K], T h, int lane, int D) {
  const int q = D >= 0 ? D / K : -1;  // source lane offset
  const int j = D - q * K;            // element of the source lane
  if (q == 0) return w[j];
  const int src = min(max(lane + q, 0), 63);
  T v = __shfl(w[j], src, 64);
  if (q < 0) {
    const T hv = readlane_t(h, 3 + D);  // lane 0 needs run cell D in [-2, -1]
    v = lane == 0 ? hv : v;
  } else {
#pragma unroll
    for (int L = 64 - q; L < 64; ++L) {
      const int t = L * K + D - 64 * K;  // 0 .. 2: run cell 64K + t
      const T hv = readlane_t(h, 3 + t);
      v = lane == L ? hv : v;
    }
  }
  return v;
}

// Load K consecutive elements starting at p (16-byte vector loads when `vec`).
template <int K, typename T>
__device__ __forceinline__ void load_run(const T* p, T (&d)[K], bool vec) {
  if constexpr (sizeof(T) == 8 && K % 2 == 0) {
    if (vec) {
#pragma unroll
      for (int j = 0; j < K / 2; ++j) {
        const double2 t = reinterpret_cast<const double2*>(p)[j];
        d[2 * j] = t.x;
        d[2 * j + 1] = t.y;
      }
      return;
    }
  }
  if constexpr (sizeof(T) == 4 && K % 4 == 0) {
    if (vec) {
#pragma unroll
      for (int j = 0; j < K / 4; ++j) {
        const float4 t = reinterpret_cast<const float4*>(p)[j];
        d[4 * j] = t.x;
        d[4 * j + 1] = t.y;
        d[4 * j + 2] = t.z;
        d[4 * j + 3] = t.w;
      }
      return;
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j) d[j] = p[j];
}

template <int K, typename T>
__device__ __forceinline__ void store_run(T* p, const T (&d)[K], bool vec) {
  if constexpr (sizeof(T) == 8 && K % 2 == 0) {
    if (vec) {
#pragma unroll
      for (int j = 0; j < K / 2; ++j)
        reinterpret_cast<double2*>(p)[j] = make_double2(d[2 * j], d[2 * j + 1]);
      return;
    }
  }
  if constexpr (sizeof(T) == 4 && K % 4 == 0) {
    if (vec) {
#pragma unroll
      for (int j = 0; j < K / 4; ++j)
        reinterpret_cast<float4*>(p)[j] =
            make_float4(d[4 * j], d[4 * j + 1], d[4 * j + 2], d[4 * j + 3]);
      return;
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j) p[j] = d[j];
}

// Evaluate the run of 64*K cells starting at cell g0 of the row at element `rowoff` of every
// component plane (cells >= n of a ragged last run are neither stored nor reduced).  Called by
// all 64 lanes of a wave with the same arguments.  SPEED: fold max(|u| + c) of the output
// cells into smax (lane-local; the caller reduces).
template <int K, int SYS, typename T, bool SPEED>
__device__ __forceinline__ void wave_run(const RowArgs<T>& a, int64_t g0, int64_t rowoff,
                                         T alpha, double dt, double& smax) {
  static_assert(K >= 2 && 64 * K >= 6, "wave run needs K >= 2");
  constexpr int NV = SysInfo<SYS>::NV;
  constexpr int TT = 64 * K;
  const int lane = threadIdx.x & 63;
  const int64_t n = a.n;
  const T gm1 = T(a.gamma) - T(1);
  const T adv = T(a.adv);
  const bool full = g0 + TT <= n;  // every own cell is a row cell (wave-uniform)
  const int64_t c0 = g0 + (int64_t)lane * K;

  // ---- load the own cells and the halo cell
  T U[NV][K], Uh[NV];
  {
    const int hp = lane < 3 ? lane - 3 : TT + lane - 3;  // halo run cell of lanes 0..5
    const int64_t hi = rowoff + bc_index(g0 + hp, n, a.bc);
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      const T* base = a.uin + c * a.plane + rowoff;
      if (full) {
        const bool vec = ((uintptr_t)(base + g0) & 15) == 0;
        load_run<K, T>(base + c0, U[c], vec);
      } else {
#pragma unroll
        for (int j = 0; j < K; ++j) U[c][j] = base[bc_index(c0 + j, n, a.bc)];
      }
      Uh[c] = lane < 6 ? a.uin[c * a.plane + hi] : U[c][0];
    }
  }

  // ---- velocity and pressure of the own and halo cells (Euler)
  T uu[K + 1], pp[K + 1];
  if constexpr (SYS == SYS_EULER1) {
#pragma unroll
    for (int j = 0; j <= K; ++j) {
      const T rho = j < K ? U[0][j] : Uh[0], m = j < K ? U[1][j] : Uh[1];
      const T E = j < K ? U[2][j] : Uh[2];
      euler1_prim<T>(rho, m, E, gm1, uu[j], pp[j]);
    }
  }

  const T eps_s = T(a.eps_s), A = window_const<T>(a.A);
  const T coef = T(-0.5 / a.dx);
  T O[NV][K];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    // U^n of the stage combination, issued early
    T Un[K];
    if (a.mode == MODE_STAGE && a.un) {
      const T* base = a.un + c * a.plane + rowoff;
      if (full) load_run<K, T>(base + c0, Un, ((uintptr_t)(base + g0) & 15) == 0);
      else
#pragma unroll
        for (int j = 0; j < K; ++j) Un[j] = base[c0 + j < n ? c0 + j : n - 1];
    }
    // split fluxes of component c
    T wp[K], wm[K], hpw, hmw;
#pragma unroll
    for (int j = 0; j <= K; ++j) {
      T Fc;
      const T Uc = j < K ? U[c][j] : Uh[c];
      if constexpr (SYS == SYS_ADV) {
        Fc = adv * Uc;
      } else {
        const T m = j < K ? U[1][j] : Uh[1], E = j < K ? U[2][j] : Uh[2];
        Fc = euler1_flux_comp<T>(c, m, E, uu[j], pp[j]);
      }
      const T p = fma_t(alpha, Uc, Fc), q = fma_t(-alpha, Uc, Fc);
      if (j < K) { wp[j] = p; wm[j] = q; }
      else { hpw = p; hmw = q; }
    }
    // windows: w^+ at run cells lK-2 .. lK+K+1; w^- mirrored, lK+K+2 down to lK-1
    T fh[K];
    {
      T v[K + 4], h[K];
#pragma unroll
      for (int i = 0; i < K + 4; ++i) v[i] = run_cell<K, T>(wp, hpw, lane, i - 2);
      wzn_window<K>(v, h, eps_s, A);
#pragma unroll
      for (int m = 0; m < K; ++m) fh[m] = h[m];
#pragma unroll
      for (int i = 0; i < K + 4; ++i) v[i] = run_cell<K, T>(wm, hmw, lane, K + 2 - i);
      wzn_window<K>(v, h, eps_s, A);
#pragma unroll
      for (int m = 0; m < K; ++m) fh[m] += h[K - 1 - m];
    }
    // the run's left boundary interface: lane 0 reconstructs w^+ at cells -3..1, lane 1 the
    // mirrored w^- at cells 2..-2 (every lane evaluates; two results are used)
    T fl0;
    {
      T v[5], h[1];
      const bool pl = lane == 0;
      v[0] = pl ? readlane_t(hpw, 0) : readlane_t(wm[2 % K], 2 / K);
      v[1] = pl ? readlane_t(hpw, 1) : readlane_t(wm[1 % K], 1 / K);
      v[2] = pl ? readlane_t(hpw, 2) : readlane_t(wm[0], 0);
      v[3] = pl ? readlane_t(wp[0], 0) : readlane_t(hmw, 2);
      v[4] = pl ? readlane_t(wp[1 % K], 1 / K) : readlane_t(hmw, 1);
      wzn_window<1>(v, h, eps_s, A);
      const T ex = readlane_t(h[0], 0) + readlane_t(h[0], 1);
      const T prev = __shfl(fh[K - 1], max(lane - 1, 0), 64);
      fl0 = lane == 0 ? ex : prev;
    }
    // flux difference and stage combination
    T o[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const T L = coef * (fh[m] - (m == 0 ? fl0 : fh[m - 1]));
      if (a.mode == MODE_RHS) {
        o[m] = L;
      } else {
        // the stage combination of stage_base(): fma(b_s dt, L, fma(a_s, U^n, b_s U))
        T base = T(a.rk_b) * U[c][m];
        if (a.un) base = fma_t(T(a.rk_a), Un[m], base);
        o[m] = fma_t(T(a.rk_b * dt), L, base);
      }
      O[c][m] = o[m];
    }
    T* ob = a.out + c * a.plane + rowoff;
    if (full) {
      store_run<K, T>(ob + c0, o, ((uintptr_t)(ob + g0) & 15) == 0);
    } else {
#pragma unroll
      for (int m = 0; m < K; ++m)
        if (c0 + m < n) ob[c0 + m] = o[m];
    }
  }
  if constexpr (SPEED && SYS == SYS_EULER1) {
#pragma unroll
    for (int m = 0; m < K; ++m) {
      if (c0 + m < n) {
        const double S[3] = {double(O[0][m]), double(O[1][m]), double(O[2][m])};
        smax = fmax(smax, wave_speed_1d<SYS>(S, a.adv, a.gamma));
      }
    }
  }
}

}  // namespace wzn
