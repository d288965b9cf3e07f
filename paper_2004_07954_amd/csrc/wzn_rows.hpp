// Arguments of the row kernel (1D right-hand side / RK stage, 2D x sweep).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wzn_host.hpp"

namespace wzn {

enum { SYS_ADV = 0, SYS_EULER1 = 1, SYS_EULER2X = 2 };
enum { MODE_RHS = 0, MODE_STAGE = 1 };
enum { SPLIT_LF = 0, SPLIT_SW = 1 };  // flux splitting (the values of wzn_params.flux_split)

template <typename T>
struct RowArgs {
  const T* uin;        // stage input U^(s): component c, row j, cell i at c*plane + j*row_stride + i
  const T* un;         // U^n for the stage combination, or null when a_s == 0
  T* out;              // L (MODE_RHS) or U^(s+1) (MODE_STAGE), same layout
  int64_t n;           // cells per row
  int64_t plane;       // elements per component
  int64_t row_stride;  // elements between rows
  double dx;
  int bc;
  int mode;
  int split;           // SPLIT_LF, or SPLIT_SW (2D x sweep only; alpha is then unused)
  int weights;         // WEIGHTS_ZN, or WEIGHTS_Z (1D fp64 only)
  // slab of a longer 1D row (one GPU's share): its three cells below and above come from
  // these [nvar][3] arrays instead of the boundary condition (1D Euler right-hand side only)
  const T* ghost_lo;
  const T* ghost_hi;
  double rk_a, rk_b;
  double adv, gamma, eps_s, A;
  double inv_gamma, inv_gm1;  // 1 / gamma, 1 / (gamma - 1) (Steger-Warming split)
  // LF alpha of this RHS evaluation: slot (reduced) / array (frozen) / constant
  const unsigned long long* alpha_slot;
  const double* alpha_arr;
  double alpha_const;
  // dt: array / cfl dx / (speed in a slot) / the dt slot
  const double* dt_arr;
  const unsigned long long* dt_speed_slot;
  const double* dt_slot_read;
  double cfl;
  double* dt_slot_write;
  double* dt_rec;
  double* alpha_rec;
  // epilogue (1D only)
  unsigned long long* speed_next;  // atomic max of |u| + c of the output, or null
  unsigned long long* slot_zero;   // zeroed by workgroup (0,0), or null
};

int launch_rows(const RowArgs<double>& a, int sys, int64_t rows, const Tuning1D& tn,
                hipStream_t s);
int launch_rows(const RowArgs<float>& a, int sys, int64_t rows, const Tuning1D& tn,
                hipStream_t s);

}  // namespace wzn
