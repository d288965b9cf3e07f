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
// layout (position p -> (p mod K) * LD + p / K) so that lane t writing or reading position
// t*K + m hits consecutive words for every m.
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

// Twice the Steger-Warming split flux, w = 2 F^{+-} (Sec. 4.4 cites the splitting), of a 2D
// Euler state along x (DIR = 0: normal velocity u, tangential v) or y (DIR = 1), for the sign
// NEG = false (+) or true (-).  With the eigenvalues (un - c, un, un + c) split as
// l^{+-} = max(l, 0) / min(l, 0) (the same bits as (l +- |l|) / 2), S = l1 + l4, Dl = l4 - l1,
// s0 = 2 (gamma - 1) l2 + S and k = rho / gamma, the ideal-gas form
//   w = k (s0, un s0 + c Dl [normal], ut s0 [tangential], q2 s0 / 2 + c (S c / (gamma - 1) + un Dl))
// (q2 = u^2 + v^2) is the textbook F^{+-} = rho/(2 gamma) (...) with the energy terms collected.
template <int DIR, bool NEG, typename T>
__device__ __forceinline__ void sw_flux2(const T* U, T (&w)[4], T gm1, T gam, T inv_gamma,
                                         T inv_gm1) {
#pragma clang fp contract(off)
  const T rho = U[0];
  const T r = rcp_nr(rho);
  const T u = U[1] * r, v = U[2] * r;
  const T p = gm1 * fma_t(-(T(0.5) * U[2]), v, fma_t(-(T(0.5) * U[1]), u, U[3]));
  const T c = sqrt_gs((gam * p) * r);
  const T un = DIR == 0 ? u : v, ut = DIR == 0 ? v : u;
  const T l1 = NEG ? fmin(un - c, T(0)) : fmax(un - c, T(0));
  const T l2 = NEG ? fmin(un, T(0)) : fmax(un, T(0));
  const T l4 = NEG ? fmin(un + c, T(0)) : fmax(un + c, T(0));
  const T S = l1 + l4, Dl = l4 - l1;
  const T s0 = fma_t(T(2) * gm1, l2, S);
  const T k = rho * inv_gamma;
  const T q2 = fma_t(u, u, v * v);
  w[0] = k * s0;
  const T wn = k * fma_t(un, s0, c * Dl);
  const T wt = k * (ut * s0);
  w[1] = DIR == 0 ? wn : wt;
  w[2] = DIR == 0 ? wt : wn;
  w[3] = k * fma_t(T(0.5) * q2, s0, c * fma_t(S * c, inv_gm1, un * Dl));
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

// Boundary conditions as an index map (Sec. 4.2, eq:26) for an in-row cell index g in
// [-3, n + 2] (harmlessly clamped beyond): periodic wrap or transmissive copy of the edge cell.
// Row lengths are below 2^31 (checked by the host).
__device__ __forceinline__ int bc_cell(int g, int n, int bc) {
  if (bc == 0) g = g < 0 ? g + n : (g >= n ? g - n : g);
  return min(max(g, 0), n - 1);
}

// TVD-RK3 stage combination (Sec. 4) out = a_s U^n + b_s (U + dt L), evaluated as
// fma(b_s dt, L, base) with base = fma(a_s, U^n, b_s U) (base = U in the first stage, where
// a_s = 0, b_s = 1 and no U^n is read).  `ok` = false skips the U^n read (cells past the row).
template <typename T>
__device__ __forceinline__ T stage_base(const RowArgs<T>& a, T U, const T* un, bool ok) {
  const T b = T(a.rk_b) * U;
  if (!a.un) return b;
  const T v = ok ? *un : T(0);
  return fma_t(T(a.rk_a), v, b);
}

// K consecutive elements from p (16-byte vector accesses when `vec`).
template <int K, typename T>
__device__ __forceinline__ void load_run(const T* p, T (&d)[K], bool vec) {
  if constexpr (sizeof(T) == 8 && K % 2 == 0) {
    if (vec) {
      typedef double v2d __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int j = 0; j < K / 2; ++j) {
        const v2d t = reinterpret_cast<const v2d*>(p)[j];
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

// Stores are non-temporal (streaming): the stage output is not re-read by this kernel, and
// lines that stay dirty in L2 must be written back when the kernel ends.
template <int K, typename T>
__device__ __forceinline__ void store_run(T* p, const T (&d)[K], bool vec) {
  if constexpr (sizeof(T) == 8 && K % 2 == 0) {
    if (vec) {
      typedef double v2d __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int j = 0; j < K / 2; ++j) {
        const v2d t = {d[2 * j], d[2 * j + 1]};
        __builtin_nontemporal_store(t, reinterpret_cast<v2d*>(p) + j);
      }
      return;
    }
  }
  if constexpr (sizeof(T) == 4 && K % 4 == 0) {
    if (vec) {
      typedef float v4f __attribute__((ext_vector_type(4)));
#pragma unroll
      for (int j = 0; j < K / 4; ++j) {
        const v4f t = {d[4 * j], d[4 * j + 1], d[4 * j + 2], d[4 * j + 3]};
        __builtin_nontemporal_store(t, reinterpret_cast<v4f*>(p) + j);
      }
      return;
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j) __builtin_nontemporal_store(d[j], p + j);
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
// sign at a time (SPLIT = true: w^+ is staged and reconstructed, then every slot is turned into
// w^- = w^+ - 2 alpha U in place and reconstructed; half the footprint).
template <int NT, int K, int SYS, typename T, bool SPLIT = false>
constexpr size_t tile_lds_bytes() {
  return sizeof(T) * (size_t)((SPLIT ? 1 : 2) * SysInfo<SYS>::NV) * Tile<NT, K>::SZ;
}

// LDS elements of the small per-tile array EX: 2*NV boundary interface values, 6*NV halo-cell
// states (second phase of the split layout) and NV per wave (last interface flux of the wave).
template <int SYS, int NT>
constexpr int tile_ex_elems() { return (8 + NT / 64) * SysInfo<SYS>::NV; }

// Process the tile whose local cell 0 is cell g0 of the row starting at element `rowoff` of
// every component plane.  Thread t loads, reconstructs and stores the K consecutive local cells
// tK .. tK+K-1 (threads 0..5 also stage one halo cell each); split fluxes are staged in LDS at
// position p = local cell + 3.  The left interface flux of a thread's first cell is the last
// interface of the previous lane (cross-lane permute), of the previous wave (LDS) or, for the
// tile's first cell, the boundary interface.  W: dynamic LDS of tile_lds_bytes(); EX: LDS of
// tile_ex_elems() elements.  All threads of the workgroup must call it (it contains barriers).
// Element (component c, in-row cell g in [-3, n + 2]) of the stage input: the boundary
// condition's index map, or (GHOST) the caller's ghost cells of a slab of a longer row (cells
// -3..-1 from ghost_lo, n..n+2 from ghost_hi, [nvar][3] each).  Cells past n + 2 only feed
// interfaces of cells that are not stored.
template <bool GHOST, typename T>
__device__ __forceinline__ T row_elem(const RowArgs<T>& a, int c, int g, int n, int64_t rowoff) {
  if constexpr (GHOST) {
    if (g < 0) return a.ghost_lo[c * 3 + g + 3];
    if (g >= n) return a.ghost_hi[c * 3 + min(g - n, 2)];
    return a.uin[c * a.plane + rowoff + g];
  } else {
    return a.uin[c * a.plane + rowoff + bc_cell(g, n, a.bc)];
  }
}

// The states a thread of a tile works on: its K own cells and (threads 0..5) one halo cell.
template <int K, int NV, typename T>
struct TileRegs {
  T U[K][NV];
  T Uh[NV];
};

// Issue the loads of a tile's states into registers (the tile whose local cell 0 is cell g0 of
// the row at element `rowoff` of every component plane).  A persistent kernel issues the next
// tile's loads before it processes the current tile, so that they are in flight meanwhile.
template <int NT, int K, int SYS, typename T, bool GHOST = false>
__device__ __forceinline__ void tile_load(const RowArgs<T>& a, int64_t g0l, int64_t rowoff,
                                          TileRegs<K, SysInfo<SYS>::NV, T>& r) {
  constexpr int NV = SysInfo<SYS>::NV;
  constexpr int TT = NT * K;
  const int tid = threadIdx.x;
  const int n = (int)a.n;
  const int g0 = (int)g0l;
  const int c0 = g0 + tid * K;
  const bool full = g0 + TT <= n;
  // the halo cells -3, -2, -1, T, T+1, T+2 of threads 0..5 first, so that their loads are in
  // flight together with the own cells'
  if (tid < 6) {
    const int hp = tid < 3 ? tid : TT + tid;
#pragma unroll
    for (int c = 0; c < NV; ++c) r.Uh[c] = row_elem<GHOST, T>(a, c, g0 + hp - 3, n, rowoff);
  }
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    const T* up = a.uin + c * a.plane + rowoff;
    T u[K];
    if (full) {
      load_run<K, T>(up + c0, u, ((uintptr_t)(up + g0) & 15) == 0);
    } else {
#pragma unroll
      for (int j = 0; j < K; ++j) u[j] = row_elem<GHOST, T>(a, c, c0 + j, n, rowoff);
    }
#pragma unroll
    for (int j = 0; j < K; ++j) r.U[j][c] = u[j];
  }
}

template <int NT, int K, int SYS, typename T, bool SPEED, bool SPLIT = false, bool SW = false,
          int WT = WEIGHTS_ZN, bool GHOST = false, bool PRE = false>
__device__ __forceinline__ void row_tile(const RowArgs<T>& a, int64_t g0l, int64_t rowoff,
                                         T alpha, double dt, T* W, T* EX, double& smax,
                                         const TileRegs<K, SysInfo<SYS>::NV, T>* pre = nullptr) {
  static_assert(!SW || SYS == SYS_EULER2X, "the Steger-Warming split is for the 2D x sweep");
  using TL = Tile<NT, K>;
  constexpr int TT = TL::T;
  constexpr int NV = SysInfo<SYS>::NV;
  constexpr int NS = SPLIT ? 1 : 2;   // signs staged per phase
  constexpr int NPH = SPLIT ? 2 : 1;  // phases
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = (int)a.n;
  const int g0 = (int)g0l;
  const T gm1 = T(a.gamma) - T(1);
  const T adv = T(a.adv);
  const T eps_s = T(a.eps_s), A = window_const<T>(a.A);
  const T m2a = -T(2) * alpha;
  const T gam = T(a.gamma), inv_gam = T(a.inv_gamma), inv_gm1 = T(a.inv_gm1);
  const int c0 = g0 + tid * K;          // first own cell
  const bool full = g0 + TT <= n;       // every own cell is a row cell (uniform)
  T* HU = EX + 2 * NV;                  // [6][NV] halo cells' U
  T* XF = EX + 8 * NV;                  // [NT/64][NV] last interface flux of each wave

  T Ureg[K][NV];
  T fh[NV][K];
#pragma unroll
  for (int ph = 0; ph < NPH; ++ph) {
    __syncthreads();  // LDS is free (previous tile or phase has finished reading it)
    if (ph == 0) {
      // ---- own cells: load, flux, split.  w^+ = F + alpha U, w^- = w^+ - 2 alpha U in every
      //      layout, so that the split layout forms w^- from the staged w^+ with the same bits.
      //      The halo cells -3, -2, -1, T, T+1, T+2 of threads 0..5 are loaded first, so that
      //      their loads are in flight together with the own cells'.
      // (PRE: the caller has issued these loads into *pre, see tile_load)
      TileRegs<K, NV, T> ld;
      if constexpr (!PRE) tile_load<NT, K, SYS, T, GHOST>(a, g0l, rowoff, ld);
      const TileRegs<K, NV, T>& r = PRE ? *pre : ld;
      T Uh[NV];
      const int hp = tid < 3 ? tid : TT + tid;
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        Uh[c] = r.Uh[c];
#pragma unroll
        for (int j = 0; j < K; ++j) Ureg[j][c] = r.U[j][c];
      }
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int q = tpos<NT, K>(3 + tid * K + j);
        if constexpr (SW) {
          T wp[NV], wm[NV];
          sw_flux2<0, false, T>(Ureg[j], wp, gm1, gam, inv_gam, inv_gm1);
          if (!SPLIT) sw_flux2<0, true, T>(Ureg[j], wm, gm1, gam, inv_gam, inv_gm1);
#pragma unroll
          for (int c = 0; c < NV; ++c) {
            W[(NS * c) * TL::SZ + q] = wp[c];
            if (!SPLIT) W[(NS * c + 1) * TL::SZ + q] = wm[c];
          }
        } else {
          T F[NV];
          row_flux<SYS, T>(Ureg[j], F, adv, gm1);
#pragma unroll
          for (int c = 0; c < NV; ++c) {
            const T wp = fma_t(alpha, Ureg[j][c], F[c]);
            W[(NS * c) * TL::SZ + q] = wp;
            if (!SPLIT) W[(NS * c + 1) * TL::SZ + q] = fma_t(m2a, Ureg[j][c], wp);
          }
        }
      }
      // ---- halo cells on threads 0..5
      if (tid < 6) {
        const int p = hp;
        T U[NV], F[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) U[c] = Uh[c];
        const int q = tpos<NT, K>(p);
        if constexpr (SW) {
          T wp[NV], wm[NV];
          sw_flux2<0, false, T>(U, wp, gm1, gam, inv_gam, inv_gm1);
          if (!SPLIT) sw_flux2<0, true, T>(U, wm, gm1, gam, inv_gam, inv_gm1);
#pragma unroll
          for (int c = 0; c < NV; ++c) {
            W[(NS * c) * TL::SZ + q] = wp[c];
            if (!SPLIT) W[(NS * c + 1) * TL::SZ + q] = wm[c];
            else HU[tid * NV + c] = U[c];
          }
        } else {
          row_flux<SYS, T>(U, F, adv, gm1);
#pragma unroll
          for (int c = 0; c < NV; ++c) {
            const T wp = fma_t(alpha, U[c], F[c]);
            W[(NS * c) * TL::SZ + q] = wp;
            if (!SPLIT) W[(NS * c + 1) * TL::SZ + q] = fma_t(m2a, U[c], wp);
            else HU[tid * NV + c] = U[c];
          }
        }
      }
    } else {
      // ---- second phase of the split layout: w^- from the staged w^+ of the same slot
      //      (Lax-Friedrichs) or from the state (Steger-Warming)
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int q = tpos<NT, K>(3 + tid * K + j);
        if constexpr (SW) {
          T wm[NV];
          sw_flux2<0, true, T>(Ureg[j], wm, gm1, gam, inv_gam, inv_gm1);
#pragma unroll
          for (int c = 0; c < NV; ++c) W[c * TL::SZ + q] = wm[c];
        } else {
#pragma unroll
          for (int c = 0; c < NV; ++c)
            W[c * TL::SZ + q] = fma_t(m2a, Ureg[j][c], W[c * TL::SZ + q]);
        }
      }
      if (tid < 6) {
        const int q = tpos<NT, K>(tid < 3 ? tid : TT + tid);
        if constexpr (SW) {
          T wm[NV];
          sw_flux2<0, true, T>(HU + tid * NV, wm, gm1, gam, inv_gam, inv_gm1);
#pragma unroll
          for (int c = 0; c < NV; ++c) W[c * TL::SZ + q] = wm[c];
        } else {
#pragma unroll
          for (int c = 0; c < NV; ++c)
            W[c * TL::SZ + q] = fma_t(m2a, HU[tid * NV + c], W[c * TL::SZ + q]);
        }
      }
      if (a.mode == MODE_STAGE) {
        // U is not needed past this point: replace it by the stage base a_s U^n + b_s U (the
        // U^n read is issued here, mid-kernel, rather than in the epilogue).  All U^n loads
        // are issued before any is combined: the register pins below would otherwise wait
        // for each load before issuing the next.
        T unv[NV][K];
        if (a.un) {
#pragma unroll
          for (int c = 0; c < NV; ++c) {
            const T* unp = a.un + c * a.plane + rowoff;
            if (full) {
              load_run<K, T>(unp + c0, unv[c], ((uintptr_t)(unp + g0) & 15) == 0);
            } else {
#pragma unroll
              for (int j = 0; j < K; ++j) unv[c][j] = c0 + j < n ? unp[c0 + j] : T(0);
            }
          }
        }
        // (a.un is uniform: a branch around both forms, not a select per value)
        if (a.un) {
#pragma unroll
          for (int c = 0; c < NV; ++c) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
              Ureg[j][c] = fma_t(T(a.rk_a), unv[c][j], T(a.rk_b) * Ureg[j][c]);
              asm volatile("" : "+v"(Ureg[j][c]));  // combine here, not in the epilogue
            }
          }
        } else {
#pragma unroll
          for (int c = 0; c < NV; ++c) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
              Ureg[j][c] = T(a.rk_b) * Ureg[j][c];
              asm volatile("" : "+v"(Ureg[j][c]));
            }
          }
        }
      }
    }
    __syncthreads();
    if (SPLIT && ph == 0 && a.mode == MODE_STAGE && a.un) {
      // warm the caches with this thread's U^n lines, read in the second phase: direct-to-LDS
      // loads into a scratch area that is never read, so no registers are held while the
      // first phase's windows run
      __shared__ int PF[NT];
      const int cc = c0 < n ? c0 : n - 1;
#pragma unroll
      for (int c = 0; c < NV; ++c)
        __builtin_amdgcn_global_load_lds(
            (const void*)(a.un + c * a.plane + rowoff + cc),
            (__attribute__((address_space(3))) void*)(PF + wave * 64), 4, 0, 0);
    }

    // ---- left boundary interface of the tile: one (component, sign) per lane
    if (tid < NS * NV) {
      const int c = tid / NS, sg = SPLIT ? ph : (tid & 1);
      T v[5], h[1];
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        const int p = sg == 0 ? i : 5 - i;  // w^+ at cells -3..1; w^- mirrored, cells 2..-2
        v[i] = W[(NS * c + (SPLIT ? 0 : sg)) * TL::SZ + tpos<NT, K>(p)];
      }
      wzn_window<1, WT>(v, h, eps_s, A);
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
        wzn_window<K, WT>(v, h, eps_s, A);
#pragma unroll
        for (int m = 0; m < K; ++m) {
          fh[c][m] = h[m];
          // materialise here: otherwise the compiler sinks the last steps of the window past
          // the following barriers and keeps the window values alive across them
          asm volatile("" : "+v"(fh[c][m]));
        }
      }
      if (!SPLIT || ph == 1) {
        // w^- mirrored: r[i] = w^- at position tK + K + 5 - i (local cell tK + K + 2 - i)
#pragma unroll
        for (int i = 0; i < K + 4; ++i) {
          const int pp = K + 5 - i;
          v[i] = W[(NS * c + NS - 1) * TL::SZ + (pp % K) * TL::LD + tid + pp / K];
        }
        wzn_window<K, WT>(v, h, eps_s, A);
#pragma unroll
        for (int m = 0; m < K; ++m) {
          fh[c][m] += h[K - 1 - m];
          asm volatile("" : "+v"(fh[c][m]));
        }
      }
    }
  }

  // ---- left interface flux of the thread's first cell
  if (lane == 63) {
#pragma unroll
    for (int c = 0; c < NV; ++c) XF[wave * NV + c] = fh[c][K - 1];
  }
  __syncthreads();
  T fl0[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    const T prev = lane_prev(fh[c][K - 1]);
    fl0[c] = lane != 0 ? prev
                       : (wave == 0 ? EX[2 * c] + EX[2 * c + 1] : XF[(wave - 1) * NV + c]);
  }

  // ---- flux difference, stage combination, store, wave speed of the output
  const T coef = T(-0.5 / a.dx);
  const T cdt = T(a.rk_b * dt);
  T O[NV][K];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    T o[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const T L = coef * (fh[c][m] - (m == 0 ? fl0[c] : fh[c][m - 1]));
      if (a.mode == MODE_RHS) {
        o[m] = L;
      } else {
        const T base = SPLIT ? Ureg[m][c]
                             : stage_base<T>(a, Ureg[m][c],
                                             a.un ? a.un + c * a.plane + rowoff + c0 + m : nullptr,
                                             c0 + m < n);
        o[m] = fma_t(cdt, L, base);
      }
      O[c][m] = o[m];
    }
    T* op = a.out + c * a.plane + rowoff;
    if (full) {
      store_run<K, T>(op + c0, o, ((uintptr_t)(op + g0) & 15) == 0);
    } else {
#pragma unroll
      for (int m = 0; m < K; ++m)
        if (c0 + m < n) op[c0 + m] = o[m];
    }
  }
  if constexpr (SPEED && SYS != SYS_EULER2X) {
#pragma unroll
    for (int m = 0; m < K; ++m) {
      if (full || c0 + m < n) {  // (no per-cell test in full tiles)
        double S[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) S[c] = double(O[c][m]);
        smax = fmax(smax, wave_speed_1d<SYS>(S, a.adv, a.gamma));
      }
    }
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
