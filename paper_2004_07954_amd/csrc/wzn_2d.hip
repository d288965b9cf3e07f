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
// Column kernel layout: a workgroup of NG waves walks down a strip of 64 columns (lane =
// column, so every global access of a row is coalesced), TY = NG*K rows per iteration; the
// split fluxes of the iteration's rows plus 3 halo rows above and below are staged in LDS one
// sign at a time, each thread reconstructs the upper interfaces of its K rows on a register
// window, and the interface between groups and between iterations is passed through LDS, so
// the only extra interface is the one below a segment's first row.
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
  int split;      // SPLIT_LF, or SPLIT_SW (alpha is then unused)
  int seg;        // rows per segment (a multiple of the tile height)
  double rk_a, rk_b;
  double gamma, eps_s, A;
  double inv_gamma, inv_gm1;  // 1 / gamma, 1 / (gamma - 1) (Steger-Warming split)
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
  // strip of a larger grid (one GPU's share): the three rows below and above it come from
  // these [4][3][nx] arrays (rows -3..-1 and ny..ny+2) instead of the boundary condition
  const T* ghost_lo;
  const T* ghost_hi;
};

// Column tile: NG row groups (one 64-lane wave each) of K rows, 64 columns; TY = NG*K rows per
// iteration plus 3 halo rows above and below staged in LDS.
template <int NG, int K>
struct ColTile {
  static constexpr int TY = NG * K;
  static constexpr int NPOS = TY + 6;
  // the six halo positions (0..2 above the tile, TY+3..TY+5 below) are staged by the first
  // HG groups, HPG each: one each when there are at least six groups, else two each
  static constexpr int HPG = NG >= 6 ? 1 : 2;
  static constexpr int HG = 6 / HPG;
  static __device__ __forceinline__ int halo_pos(int g, int hh) {
    if constexpr (NG >= 6) return g < 3 ? g : TY + g;
    else return hh == 0 ? g : TY + 3 + g;
  }
};

// y flux G = (rho v, rho u v, rho v^2 + p, v (E + p)) of a 2D Euler state, through one
// reciprocal of rho, in a fixed operation order.
template <typename T>
__device__ __forceinline__ void flux_y(const T (&U)[4], T (&G)[4], T gm1) {
#pragma clang fp contract(off)
  const T r = rcp_nr(U[0]);
  const T u = U[1] * r, v = U[2] * r;
  const T p = gm1 * fma_t(-(T(0.5) * U[2]), v, fma_t(-(T(0.5) * U[1]), u, U[3]));
  G[0] = U[2];
  G[1] = U[1] * v;
  G[2] = fma_t(U[2], v, p);
  G[3] = v * (U[3] + p);
}

// The state of row y in [-3, ny + 2] (rows past ny + 2 only feed interfaces of rows that are
// not stored) at column xc: the boundary condition's index map, or (GHOST) the caller's ghost
// rows below and above a strip.
template <bool GHOST, typename T>
__device__ __forceinline__ void col_state(const ColArgs<T>& a, int y, int ny, int nx, int xc,
                                          T (&U)[4]) {
  if constexpr (GHOST) {
    if (y < 0 || y >= ny) {
      const T* gsrc = y < 0 ? a.ghost_lo : a.ghost_hi;
      const int r = y < 0 ? y + 3 : min(y - ny, 2);
#pragma unroll
      for (int c = 0; c < 4; ++c) U[c] = gsrc[((int64_t)c * 3 + r) * nx + xc];
      return;
    }
    const int64_t gi = (int64_t)y * nx + xc;
#pragma unroll
    for (int c = 0; c < 4; ++c) U[c] = a.uin[c * a.plane + gi];
  } else {
    const int64_t gi = (int64_t)bc_cell(y, ny, a.bc) * nx + xc;
#pragma unroll
    for (int c = 0; c < 4; ++c) U[c] = a.uin[c * a.plane + gi];
  }
}

// One workgroup walks down the rows [y_s, y_e) of a strip of 64 columns, TY rows per iteration.
// Thread (column, group g) loads, reconstructs and finishes rows y0 + gK .. y0 + gK + K - 1 of
// its column; the split fluxes of all components are staged one sign at a time (w^+ first,
// then w^- = w^+ - 2 alpha U in place).  The lower interface of a group's first row is the
// last interface of the group below (LDS), of the previous iteration's last group (carried in
// LDS), or at the segment's first row the boundary interface, reconstructed once per segment.
// Two register budgets:
//  - four waves per SIMD (128 VGPRs): the state of the next iteration is loaded after the
//    finish, and Lx and U^n of all components are loaded together before the second phase's
//    windows;
//  - (PF, the fp64 Steger-Warming split, whose flux arithmetic needs more registers) three
//    waves per SIMD (168 VGPRs): the next iteration's state is loaded before the finish, and
//    each component's Lx and U^n one window ahead, so that their latency overlaps arithmetic.
template <typename T, bool SW>
struct ColPrefetch {
  static constexpr bool value = SW && sizeof(T) == 8;
};
template <int NG, int K, typename T, bool SPEED, bool SW, bool GHOST>
__global__ __launch_bounds__(64 * NG)
__attribute__((amdgpu_waves_per_eu(ColPrefetch<T, SW>::value ? 3 : 4)))
void col_kernel(ColArgs<T> a) {
  static_assert(NG >= 4, "the segment's boundary interface uses one group per component");
  constexpr bool PF = ColPrefetch<T, SW>::value;
  using CT = ColTile<NG, K>;
  constexpr int TY = CT::TY, NPOS = CT::NPOS;
  __shared__ T W[4 * NPOS * 64];
  __shared__ T XF[(NG - 1) * 4 * 64];
  __shared__ T CARRY[2][4 * 64];
  __shared__ double red[2][NG];
  const int col = threadIdx.x & 63;
  // the row group is the wave index: uniform across the wave, so held in a scalar register
  // (the group branches below are then scalar branches, not exec masks)
  const int g = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nx = (int)a.nx, ny = (int)a.ny;
  const int x = blockIdx.x * 64 + col;
  const bool xin = x < nx;
  const int xc = xin ? x : nx - 1;
  const int ys = blockIdx.y * a.seg;
  const int ye = min(ys + a.seg, ny);

  double alpha_d;
  if (a.alpha_slot) alpha_d = slot_value(a.alpha_slot);
  else if (a.alpha_arr) alpha_d = a.alpha_arr[0];
  else alpha_d = a.alpha_const;
  const T alpha = T(alpha_d);
  const T m2a = -T(2) * alpha;
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
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    if (a.dt_slot_write) a.dt_slot_write[0] = dt;
    if (a.dt_rec) a.dt_rec[0] = dt;
    if (a.zero_x) a.zero_x[0] = 0ull;
    if (a.zero_y) a.zero_y[0] = 0ull;
  }

  const T gm1 = T(a.gamma) - T(1);
  const T gam = T(a.gamma), inv_gam = T(a.inv_gamma), inv_gm1 = T(a.inv_gm1);
  const T eps_s = T(a.eps_s), A = window_const<T>(a.A);
  const T coef = T(-0.5 / a.dy);
  const T cdt = a.mode == MODE_STAGE ? T(a.rk_b * dt) : T(1);
  const double gamma = a.gamma;
  double sxm = 0.0, sym = 0.0;

  T Ureg[K][4];   // own rows: state, then (second phase) the base of the output
  T HU[CT::HPG][4];  // halo rows staged by this group (groups below CT::HG)
  T fh[4][K];
  // the state of the group's own rows and halo rows of the iteration starting at row y0
  auto load_rows = [&](int y0, T (&Ur)[K][4], T (&Hr)[CT::HPG][4]) {
#pragma unroll
    for (int j = 0; j < K; ++j) col_state<GHOST, T>(a, y0 + g * K + j, ny, nx, xc, Ur[j]);
    if (g < CT::HG) {
#pragma unroll
      for (int hh = 0; hh < CT::HPG; ++hh)
        col_state<GHOST, T>(a, y0 + CT::halo_pos(g, hh) - 3, ny, nx, xc, Hr[hh]);
    }
  };
  // Lx and U^n of component c of the group's own rows (rows past the segment read the
  // segment's first row instead: every load is in bounds, and those rows are never stored)
  auto load_base = [&](int y0, int c, T (&lx)[K], T (&un)[K]) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int y = y0 + g * K + j;
      const int64_t gi = (int64_t)(y < ye ? y : ys) * nx + xc;
      lx[j] = a.lx[c * a.plane + gi];
      un[j] = a.mode == MODE_STAGE && a.un ? a.un[c * a.plane + gi] : T(0);
    }
  };
  // replace the state of component c by the base of the output: Lx (RHS) or
  // fma(b_s dt, Lx, fma(a_s, U^n, b_s U)) (stage), so that the output is fma(cdt, Ly, base)
  // with cdt = 1 or b_s dt
  auto combine = [&](int c, const T (&lx)[K], const T (&un)[K]) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      T base = lx[j];
      if (a.mode == MODE_STAGE) {
        T b = T(a.rk_b) * Ureg[j][c];
        if (a.un) b = fma_t(T(a.rk_a), un[j], b);
        base = fma_t(cdt, lx[j], b);
      }
      Ureg[j][c] = base;
      asm volatile("" : "+v"(Ureg[j][c]));  // combine here, not in the epilogue
    }
  };
  if (ys < ye) load_rows(ys, Ureg, HU);
  int it = 0;
  for (int y0 = ys; y0 < ye; y0 += TY, ++it) {
    const int par = it & 1;
#pragma unroll
    for (int ph = 0; ph < 2; ++ph) {
      __syncthreads();  // W, XF and CARRY of the previous phase / iteration are consumed
      if (ph == 0) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
          T G[4];
          const int p = 3 + g * K + j;
          if constexpr (SW) {
            sw_flux2<1, false, T>(Ureg[j], G, gm1, gam, inv_gam, inv_gm1);
#pragma unroll
            for (int c = 0; c < 4; ++c) W[(c * NPOS + p) * 64 + col] = G[c];
          } else {
            flux_y<T>(Ureg[j], G, gm1);
#pragma unroll
            for (int c = 0; c < 4; ++c) W[(c * NPOS + p) * 64 + col] = fma_t(alpha, Ureg[j][c], G[c]);
          }
        }
        if (g < CT::HG) {
#pragma unroll
          for (int hh = 0; hh < CT::HPG; ++hh) {
            const int p = CT::halo_pos(g, hh);
            T G[4];
            if constexpr (SW) {
              // (the second phase re-reads the halo state rather than holding it)
              sw_flux2<1, false, T>(HU[hh], G, gm1, gam, inv_gam, inv_gm1);
#pragma unroll
              for (int c = 0; c < 4; ++c) W[(c * NPOS + p) * 64 + col] = G[c];
            } else {
              flux_y<T>(HU[hh], G, gm1);
#pragma unroll
              for (int c = 0; c < 4; ++c) W[(c * NPOS + p) * 64 + col] = fma_t(alpha, HU[hh][c], G[c]);
            }
          }
        }
      } else {
        // w^- from the staged w^+ of the same slot (Lax-Friedrichs) or from the state
        // (Steger-Warming)
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const int p = 3 + g * K + j;
          if constexpr (SW) {
            T G[4];
            sw_flux2<1, true, T>(Ureg[j], G, gm1, gam, inv_gam, inv_gm1);
#pragma unroll
            for (int c = 0; c < 4; ++c) W[(c * NPOS + p) * 64 + col] = G[c];
          } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              T& w = W[(c * NPOS + p) * 64 + col];
              w = fma_t(m2a, Ureg[j][c], w);
            }
          }
        }
        if (g < CT::HG) {
#pragma unroll
          for (int hh = 0; hh < CT::HPG; ++hh) {
            const int p = CT::halo_pos(g, hh);
            if constexpr (SW) {
              T Uh[4], G[4];
              col_state<GHOST, T>(a, y0 + p - 3, ny, nx, xc, Uh);
              sw_flux2<1, true, T>(Uh, G, gm1, gam, inv_gam, inv_gm1);
#pragma unroll
              for (int c = 0; c < 4; ++c) W[(c * NPOS + p) * 64 + col] = G[c];
            } else {
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                T& w = W[(c * NPOS + p) * 64 + col];
                w = fma_t(m2a, HU[hh][c], w);
              }
            }
          }
        }
        if constexpr (!PF) {
          // (Steger-Warming: keep the loads below from being hoisted into the split arithmetic
          // above, where their registers would be live at the same time)
          if constexpr (SW) asm volatile("" ::: "memory");
          // the state is not needed past this point: all loads of the row group are issued
          // before any is combined (the register pins would otherwise wait for each load
          // before issuing the next)
          T lxv[4][K], unv[4][K];
#pragma unroll
          for (int c = 0; c < 4; ++c) load_base(y0, c, lxv[c], unv[c]);
#pragma unroll
          for (int c = 0; c < 4; ++c) combine(c, lxv[c], unv[c]);
        }
      }
      __syncthreads();

      // the segment's boundary interface (below its first row): group c < 4 reconstructs
      // component c, sign ph; carried in as the previous iteration's last interface
      if (it == 0 && g < 4) {
        T v[5], h[1];
#pragma unroll
        for (int i = 0; i < 5; ++i) v[i] = W[(g * NPOS + (ph == 0 ? i : 5 - i)) * 64 + col];
        wzn_window<1>(v, h, eps_s, A);
        if (ph == 0) CARRY[1][g * 64 + col] = h[0];
        else CARRY[1][g * 64 + col] += h[0];
      }

      // windows: thread (col, g) owns the upper interfaces of rows gK .. gK+K-1.  (PF: in
      // the second phase each component's state is replaced by the base after its window,
      // with the loads of its Lx and U^n issued one window ahead.)
      T lxq[2][K], unq[2][K];
      if (PF && ph == 1) load_base(y0, 0, lxq[0], unq[0]);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        T v[K + 4], h[K];
        if (PF && ph == 1 && c < 3) load_base(y0, c + 1, lxq[(c + 1) & 1], unq[(c + 1) & 1]);
        if (ph == 0) {
#pragma unroll
          for (int i = 0; i < K + 4; ++i) v[i] = W[(c * NPOS + g * K + 1 + i) * 64 + col];
          wzn_window<K>(v, h, eps_s, A);
#pragma unroll
          for (int m = 0; m < K; ++m) {
            fh[c][m] = h[m];
            asm volatile("" : "+v"(fh[c][m]));
          }
        } else {
#pragma unroll
          for (int i = 0; i < K + 4; ++i) v[i] = W[(c * NPOS + g * K + K + 5 - i) * 64 + col];
          wzn_window<K>(v, h, eps_s, A);
#pragma unroll
          for (int m = 0; m < K; ++m) {
            fh[c][m] += h[K - 1 - m];
            asm volatile("" : "+v"(fh[c][m]));
          }
          if constexpr (PF) combine(c, lxq[c & 1], unq[c & 1]);
        }
      }
    }
    // (PF) the next iteration's rows are loaded now: the loads are in flight during the
    // exchange and the finish below
    T Unx[K][4], HUnx[CT::HPG][4];
    const bool more = y0 + TY < ye;
    if (PF && more) load_rows(y0 + TY, Unx, HUnx);
    // ---- exchange the groups' last interfaces
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (g < NG - 1) XF[(g * 4 + c) * 64 + col] = fh[c][K - 1];
      else CARRY[par][c * 64 + col] = fh[c][K - 1];
    }
    __syncthreads();
    T fl0[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
      fl0[c] = g == 0 ? CARRY[par ^ 1][c * 64 + col] : XF[((g - 1) * 4 + c) * 64 + col];

    // ---- finish the rows: Ly, output, wave speeds
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const int y = y0 + g * K + m;
      const bool ok = y < ye && xin;
      const int64_t gi = (int64_t)(ok ? y : ys) * nx + xc;
      T o[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const T Ly = coef * (fh[c][m] - (m == 0 ? fl0[c] : fh[c][m - 1]));
        o[c] = fma_t(cdt, Ly, Ureg[m][c]);
        if (ok) __builtin_nontemporal_store(o[c], a.out + c * a.plane + gi);
      }
      if constexpr (SPEED) {
        if (ok) {
          double ax, ay;
          wave_speeds_2d(double(o[0]), double(o[1]), double(o[2]), double(o[3]), gamma, ax, ay);
          sxm = fmax(sxm, ax);
          sym = fmax(sym, ay);
        }
      }
    }
    if (!PF && more) {
      load_rows(y0 + TY, Ureg, HU);
    } else if (more) {
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int c = 0; c < 4; ++c) Ureg[j][c] = Unx[j][c];
#pragma unroll
      for (int hh = 0; hh < CT::HPG; ++hh)
#pragma unroll
        for (int c = 0; c < 4; ++c) HU[hh][c] = HUnx[hh][c];
    }
  }
  if constexpr (SPEED) {
    sxm = wave_max(sxm);
    sym = wave_max(sym);
    if (col == 0) {
      red[0][g] = sxm;
      red[1][g] = sym;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double mx = red[0][0], my = red[1][0];
#pragma unroll
      for (int w = 1; w < NG; ++w) {
        mx = fmax(mx, red[0][w]);
        my = fmax(my, red[1][w]);
      }
      atomic_max_pos(a.speed_next_x, mx);
      atomic_max_pos(a.speed_next_y, my);
    }
  }
}

template <int NG, int K, typename T>
static int launch_col_t(ColArgs<T> a, hipStream_t s) {
  constexpr int TY = ColTile<NG, K>::TY;
  const int64_t bx = (a.nx + 63) / 64;
  // Split the rows into segments (multiples of TY rows) for several rounds of resident
  // workgroups: four rounds at four waves per SIMD, eight at three (PF).  With a single round
  // the workgroups dispatched last get the smallest share of the SIMDs and finish last, so the
  // CUs drain from four resident waves per SIMD to one (measured: one round is 3-5 % slower).
  const bool pf = a.split == SPLIT_SW ? ColPrefetch<T, true>::value : ColPrefetch<T, false>::value;
  const int64_t target = pf ? 256 * 3 * 8 : 256 * 4 * 4;
  int64_t nseg = (target + bx - 1) / bx;
  const int64_t maxseg = (a.ny + TY - 1) / TY;
  if (nseg > maxseg) nseg = maxseg;
  if (nseg < 1) nseg = 1;
  int64_t seg = (a.ny + nseg - 1) / nseg;
  seg = (seg + TY - 1) / TY * TY;
  nseg = (a.ny + seg - 1) / seg;
  a.seg = (int)seg;
  if (bx > 0x7fffffff || nseg > 65535) return set_error(WZN_ERR_SIZE, "grid too large (columns)");
  const dim3 grid((unsigned)bx, (unsigned)nseg), block(64 * NG);
  if (a.ghost_lo) {  // strip right-hand side: no stage epilogue
    if (a.split == SPLIT_SW)
      hipLaunchKernelGGL((col_kernel<NG, K, T, false, true, true>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((col_kernel<NG, K, T, false, false, true>), grid, block, 0, s, a);
  } else if (a.split == SPLIT_SW) {
    if (a.speed_next_x)
      hipLaunchKernelGGL((col_kernel<NG, K, T, true, true, false>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((col_kernel<NG, K, T, false, true, false>), grid, block, 0, s, a);
  } else {
    if (a.speed_next_x)
      hipLaunchKernelGGL((col_kernel<NG, K, T, true, false, false>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((col_kernel<NG, K, T, false, false, false>), grid, block, 0, s, a);
  }
  return check_launch("col_kernel");
}

// Column kernel shape: NG row groups of K rows (K = 2 in fp64, 4 in fp32: the LDS of one
// tile, 4 * (NG K + 6) * 64 elements, stays within 40 KB for four workgroups per CU).
template <typename T> struct ColShape;
template <> struct ColShape<double> { static constexpr int NG = 4, K = 2; };
template <> struct ColShape<float> { static constexpr int NG = 4, K = 4; };

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
  a.split = p->flux_split;
  a.gamma = p->gamma;
  a.inv_gamma = 1.0 / p->gamma;
  a.inv_gm1 = 1.0 / (p->gamma - 1.0);
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
  a.split = p->flux_split;
  a.gamma = p->gamma;
  a.inv_gamma = 1.0 / p->gamma;
  a.inv_gm1 = 1.0 / (p->gamma - 1.0);
  a.eps_s = 16.0 * p->eps;
  a.A = p->A;
  return a;
}

// Launch shape of the x sweep (rows of 4 components): the process-wide row override when it
// names a shape the 2D row kernel has, else 512-cell tiles with both signs staged (measured
// fastest for 4096^2 in fp64 and fp32).
static Tuning1D tuning_2dx() {
  const Tuning1D o = row_override();
  const bool ok = (o.layout == ROW_LDS_TILE && ((o.nt == 256 && (o.k == 4 || o.k == 2)) ||
                                               (o.nt == 128 && o.k == 4))) ||
                  (o.layout == ROW_LDS_SPLIT && o.nt == 256 && (o.k == 4 || o.k == 2));
  return ok ? o : Tuning1D{256, 2, ROW_LDS_TILE};
}

template <typename T>
int rhs_2d_t(const wzn_params* p, const T* u, T* dudt, int64_t nx, int64_t ny, double dx,
             double dy, Workspace* ws, hipStream_t s) {
  RowArgs<T> ra = row_args<T>(p, nx, ny, dx);
  ColArgs<T> ca = col_args<T>(p, nx, ny, dx, dy);
  // the Steger-Warming split has no alpha
  const bool sw = p->flux_split == SPLIT_SW;
  const bool reduce = !sw && (p->lf_alpha_x < 0.0 || p->lf_alpha_y < 0.0);
  if (reduce) {
    int st = launch_zero_words(ws->speed, 6, s);
    if (st) return st;
    st = launch_speed_max<T>(u, nx * ny, 4, p->gamma, &ws->speed[0], &ws->speed_y[0], s);
    if (st) return st;
  }
  if (p->lf_alpha_x >= 0.0 || sw) ra.alpha_const = p->lf_alpha_x;
  else ra.alpha_slot = &ws->speed[0];
  if (p->lf_alpha_y >= 0.0 || sw) ca.alpha_const = p->lf_alpha_y;
  else ca.alpha_slot = &ws->speed_y[0];
  ra.uin = u;
  ra.out = dudt;
  int st = launch_rows(ra, SYS_EULER2X, ny, tuning_2dx(), s);
  if (st) return st;
  ca.uin = u;
  ca.lx = dudt;
  ca.out = dudt;
  ca.mode = MODE_RHS;
  return launch_col_t<ColShape<T>::NG, ColShape<T>::K, T>(ca, s);
}
template int rhs_2d_t<double>(const wzn_params*, const double*, double*, int64_t, int64_t, double,
                              double, Workspace*, hipStream_t);

// Right-hand side of a strip of ny rows of a larger grid (one GPU's share of a row
// decomposition): the y sweep takes its three rows below and above from ghost_lo / ghost_hi,
// and both sweeps use the caller's alphas (the maxima over the whole grid: a per-strip alpha
// would change the scheme).  The x sweep needs no halo from other strips.
template <typename T>
int rhs_2d_strip_t(const wzn_params* p, const T* u, const T* ghost_lo, const T* ghost_hi,
                   T* dudt, int64_t nx, int64_t ny, double dx, double dy, const double* alpha2,
                   hipStream_t s) {
  RowArgs<T> ra = row_args<T>(p, nx, ny, dx);
  ColArgs<T> ca = col_args<T>(p, nx, ny, dx, dy);
  ra.alpha_arr = alpha2;
  ca.alpha_arr = alpha2 ? alpha2 + 1 : nullptr;
  ra.uin = u;
  ra.out = dudt;
  int st = launch_rows(ra, SYS_EULER2X, ny, tuning_2dx(), s);
  if (st) return st;
  ca.uin = u;
  ca.lx = dudt;
  ca.out = dudt;
  ca.mode = MODE_RHS;
  ca.ghost_lo = ghost_lo;
  ca.ghost_hi = ghost_hi;
  return launch_col_t<ColShape<T>::NG, ColShape<T>::K, T>(ca, s);
}
template int rhs_2d_strip_t<double>(const wzn_params*, const double*, const double*, const double*,
                                    double*, int64_t, int64_t, double, double, const double*,
                                    hipStream_t);
template int rhs_2d_strip_t<float>(const wzn_params*, const float*, const float*, const float*,
                                   float*, int64_t, int64_t, double, double, const double*,
                                   hipStream_t);

__global__ void slots_to_doubles_kernel(const unsigned long long* sx,
                                        const unsigned long long* sy, double* out) {
  if (threadIdx.x == 0) {
    out[0] = slot_value(sx);
    out[1] = slot_value(sy);
  }
}

// max over the cells of u of |u| + c and |v| + c into out[0], out[1] (device doubles)
template <typename T>
int speed_max_2d_t(const wzn_params* p, const T* u, int64_t nx, int64_t ny, double* out,
                   Workspace* ws, hipStream_t s) {
  int st = launch_zero_words(ws->speed, 6, s);
  if (st) return st;
  st = launch_speed_max<T>(u, nx * ny, 4, p->gamma, &ws->speed[0], &ws->speed_y[0], s);
  if (st) return st;
  hipLaunchKernelGGL(slots_to_doubles_kernel, dim3(1), dim3(64), 0, s, &ws->speed[0],
                     &ws->speed_y[0], out);
  return check_launch("slots_to_doubles_kernel");
}
template int speed_max_2d_t<double>(const wzn_params*, const double*, int64_t, int64_t, double*,
                                    Workspace*, hipStream_t);
template int speed_max_2d_t<float>(const wzn_params*, const float*, int64_t, int64_t, double*,
                                   Workspace*, hipStream_t);
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
  // the Steger-Warming split has no alpha: the speed slots then serve the CFL dt only
  const bool sw = p->flux_split == SPLIT_SW;
  const bool reduce_x = !sw && p->lf_alpha_x < 0.0, reduce_y = !sw && p->lf_alpha_y < 0.0;
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
      st = launch_col_t<ColShape<T>::NG, ColShape<T>::K, T>(ca, s);
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
