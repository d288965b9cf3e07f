// Row kernel of the WENO-ZN hot path for gfx950: one workgroup per row tile (see
// wzn_tile.hpp for what a tile computes).  Used for the 1D right-hand side and fused TVD-RK3
// stages (one launch per stage; the max wave speed of the output is folded into one atomic per
// workgroup for the next stage's alpha / next step's dt) and for the x sweep of the 2D
// dimension-by-dimension right-hand side (one row per blockIdx.y).
#include <hip/hip_runtime.h>

#include "wzn_device.hpp"
#include "wzn_host.hpp"
#include "wzn_rows.hpp"
#include "wzn_tile.hpp"

namespace wzn {

// SPEED (a.speed_next set) is a template parameter rather than a branch: one kernel holding
// both inlined tile variants is register-allocated for their union.
template <int NT, int K, int SYS, typename T, bool SPLIT, bool SPEED, bool SW, int WT,
          bool GHOST>
__global__ __launch_bounds__(NT) void row_kernel(RowArgs<T> a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* W = reinterpret_cast<T*>(lds_raw);
  __shared__ T EX[tile_ex_elems<SYS, NT>()];
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x;

  // alpha and dt of this evaluation (uniform over the grid)
  double alpha_d;
  if (a.alpha_slot) alpha_d = slot_value(a.alpha_slot);
  else if (a.alpha_arr) alpha_d = a.alpha_arr[0];
  else alpha_d = a.alpha_const;
  double dt = 0.0;
  if (a.mode == MODE_STAGE) {
    if (a.dt_arr) dt = a.dt_arr[0];
    else if (a.dt_speed_slot) dt = a.cfl * a.dx / slot_value(a.dt_speed_slot);
    else dt = a.dt_slot_read[0];
  }
  if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) {
    if (a.dt_slot_write) a.dt_slot_write[0] = dt;
    if (a.dt_rec) a.dt_rec[0] = dt;
    if (a.alpha_rec) a.alpha_rec[0] = alpha_d;
    if (a.slot_zero) a.slot_zero[0] = 0ull;
  }
  const int64_t g0 = (int64_t)blockIdx.x * (NT * K);
  const int64_t rowoff = (int64_t)blockIdx.y * a.row_stride;
  double smax = 0.0;
  row_tile<NT, K, SYS, T, SPEED, SPLIT, SW, WT, GHOST>(a, g0, rowoff, T(alpha_d), dt, W, EX,
                                                       smax);
  if constexpr (SPEED) {
    const double m = block_max<NT>(smax, red);
    if (tid == 0) atomic_max_pos(a.speed_next, m);
  } else {
    (void)red;
  }
}

// ------------------------------------------------------------------ host side
template <int NT, int K, int SYS, typename T, bool SPLIT, bool SPEED, bool SW = false,
          int WT = WEIGHTS_ZN, bool GHOST = false>
static int launch_row_ts(const RowArgs<T>& a, int64_t rows, hipStream_t s) {
  constexpr int TT = NT * K;
  const int64_t blocks = (a.n + TT - 1) / TT;
  const size_t lds = tile_lds_bytes<NT, K, SYS, T, SPLIT>();
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute((const void*)row_kernel<NT, K, SYS, T, SPLIT, SPEED, SW, WT, GHOST>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return set_error(WZN_ERR_HIP, "hipFuncSetAttribute(row_kernel) failed");
    attr_set = true;
  }
  if (blocks > 0x7fffffff || rows > 65535)
    return set_error(WZN_ERR_SIZE, "grid too large for the row kernel");
  hipLaunchKernelGGL((row_kernel<NT, K, SYS, T, SPLIT, SPEED, SW, WT, GHOST>),
                     dim3((unsigned)blocks, (unsigned)rows), dim3(NT), lds, s, a);
  return check_launch("row_kernel");
}

template <int NT, int K, int SYS, typename T, bool SPLIT = false>
static int launch_row_t(const RowArgs<T>& a, int64_t rows, hipStream_t s) {
  // the wave-speed epilogue exists for the 1D Euler system only, the Steger-Warming split for
  // the 2D x sweep only
  if constexpr (SYS == SYS_EULER1) {
    if (a.speed_next) return launch_row_ts<NT, K, SYS, T, SPLIT, true>(a, rows, s);
  }
  if constexpr (SYS == SYS_EULER2X) {
    if (a.split == SPLIT_SW) return launch_row_ts<NT, K, SYS, T, SPLIT, false, true>(a, rows, s);
  }
  return launch_row_ts<NT, K, SYS, T, SPLIT, false>(a, rows, s);
}

int launch_rows(const RowArgs<double>& a, int sys, int64_t rows, const Tuning1D& tn,
                hipStream_t s) {
  if (a.ghost_lo) {
    // slab of a longer row: the 1D Euler right-hand side in one launch shape
    if (sys != SYS_EULER1 || a.mode != MODE_RHS || a.weights != WEIGHTS_ZN)
      return set_error(WZN_ERR_UNSUPPORTED, "ghost cells: 1D Euler right-hand side only");
    return launch_row_ts<256, 4, SYS_EULER1, double, true, false, false, WEIGHTS_ZN, true>(a, rows,
                                                                                           s);
  }
  if (a.weights == WEIGHTS_Z) {
    // the WENO-Z comparison weights run in one launch shape per 1D system (the tuning
    // applies to the paper's weights)
    if (sys == SYS_EULER1) {
      if (a.speed_next)
        return launch_row_ts<256, 2, SYS_EULER1, double, false, true, false, WEIGHTS_Z>(a, rows, s);
      return launch_row_ts<256, 2, SYS_EULER1, double, false, false, false, WEIGHTS_Z>(a, rows, s);
    }
    if (sys == SYS_ADV)
      return launch_row_ts<64, 4, SYS_ADV, double, false, false, false, WEIGHTS_Z>(a, rows, s);
    return set_error(WZN_ERR_UNSUPPORTED, "WENO-Z weights run in 1D only");
  }
  if (tn.layout == ROW_LDS_SPLIT) {
    if (sys == SYS_EULER1) {
      if (tn.nt == 256 && tn.k == 4) return launch_row_t<256, 4, SYS_EULER1, double, true>(a, rows, s);
      if (tn.nt == 256 && tn.k == 2) return launch_row_t<256, 2, SYS_EULER1, double, true>(a, rows, s);
      if (tn.nt == 128 && tn.k == 4) return launch_row_t<128, 4, SYS_EULER1, double, true>(a, rows, s);
      if (tn.nt == 64 && tn.k == 4) return launch_row_t<64, 4, SYS_EULER1, double, true>(a, rows, s);
      return set_error(WZN_ERR_ARG, "unsupported 1D split tuning (nt=%d, k=%d)", tn.nt, tn.k);
    }
    if (sys == SYS_EULER2X) {
      if (tn.nt == 256 && tn.k == 4) return launch_row_t<256, 4, SYS_EULER2X, double, true>(a, rows, s);
      if (tn.nt == 256 && tn.k == 2) return launch_row_t<256, 2, SYS_EULER2X, double, true>(a, rows, s);
      return set_error(WZN_ERR_ARG, "unsupported 2D-x split tuning (nt=%d, k=%d)", tn.nt, tn.k);
    }
    return set_error(WZN_ERR_ARG, "no split layout for this system");
  }
  if (sys == SYS_EULER1) {
    if (tn.nt == 256 && tn.k == 4) return launch_row_t<256, 4, SYS_EULER1, double>(a, rows, s);
    if (tn.nt == 256 && tn.k == 2) return launch_row_t<256, 2, SYS_EULER1, double>(a, rows, s);
    if (tn.nt == 128 && tn.k == 4) return launch_row_t<128, 4, SYS_EULER1, double>(a, rows, s);
    if (tn.nt == 256 && tn.k == 1) return launch_row_t<256, 1, SYS_EULER1, double>(a, rows, s);
    if (tn.nt == 128 && tn.k == 8) return launch_row_t<128, 8, SYS_EULER1, double>(a, rows, s);
    if (tn.nt == 64 && tn.k == 8) return launch_row_t<64, 8, SYS_EULER1, double>(a, rows, s);
    if (tn.nt == 64 && tn.k == 4) return launch_row_t<64, 4, SYS_EULER1, double>(a, rows, s);
    if (tn.nt == 64 && tn.k == 2) return launch_row_t<64, 2, SYS_EULER1, double>(a, rows, s);
    if (tn.nt == 64 && tn.k == 1) return launch_row_t<64, 1, SYS_EULER1, double>(a, rows, s);
    return set_error(WZN_ERR_ARG, "unsupported 1D tuning (nt=%d, k=%d)", tn.nt, tn.k);
  }
  if (sys == SYS_EULER2X) {
    if (tn.nt == 256 && tn.k == 4) return launch_row_t<256, 4, SYS_EULER2X, double>(a, rows, s);
    if (tn.nt == 128 && tn.k == 4) return launch_row_t<128, 4, SYS_EULER2X, double>(a, rows, s);
    if (tn.nt == 256 && tn.k == 2) return launch_row_t<256, 2, SYS_EULER2X, double>(a, rows, s);
    return set_error(WZN_ERR_ARG, "unsupported 2D-x tuning (nt=%d, k=%d)", tn.nt, tn.k);
  }
  return launch_row_t<64, 4, SYS_ADV, double>(a, rows, s);
}

int launch_rows(const RowArgs<float>& a, int sys, int64_t rows, const Tuning1D& tn,
                hipStream_t s) {
  if (sys != SYS_EULER2X) return set_error(WZN_ERR_DTYPE, "fp32 rows only for 2D Euler");
  if (tn.layout == ROW_LDS_SPLIT) {
    if (tn.nt == 256 && tn.k == 4) return launch_row_t<256, 4, SYS_EULER2X, float, true>(a, rows, s);
    if (tn.nt == 256 && tn.k == 2) return launch_row_t<256, 2, SYS_EULER2X, float, true>(a, rows, s);
    return set_error(WZN_ERR_ARG, "unsupported 2D-x split tuning (nt=%d, k=%d)", tn.nt, tn.k);
  }
  if (tn.nt == 256 && tn.k == 4) return launch_row_t<256, 4, SYS_EULER2X, float>(a, rows, s);
  if (tn.nt == 128 && tn.k == 4) return launch_row_t<128, 4, SYS_EULER2X, float>(a, rows, s);
  if (tn.nt == 256 && tn.k == 2) return launch_row_t<256, 2, SYS_EULER2X, float>(a, rows, s);
  return set_error(WZN_ERR_ARG, "unsupported 2D-x tuning (nt=%d, k=%d)", tn.nt, tn.k);
}

}  // namespace wzn
