// Device building blocks of the WENO-ZN hot path for gfx950 (fp64).
//
// The reconstruction is evaluated on a sliding window of K + 4 consecutive values held in
// registers, producing K consecutive interface fluxes.  Differences shared by neighbouring
// interfaces are computed once per window:
//   g_j = v_{j+1} - v_j,   D_j = g_{j+1} - g_j   (second difference centred at v_{j+1})
// and the Jiang-Shu indicators (Sec. 2.1, eq:isjiang) of interface m of the window,
// stencil (a..e) = (v_m .. v_{m+4}), are
//   IS0 = 13/12 D_m^2     + 1/4 (3 g_{m+1} - g_m)^2
//   IS1 = 13/12 D_{m+1}^2 + 1/4 (g_{m+1} + g_{m+2})^2
//   IS2 = 13/12 D_{m+2}^2 + 1/4 (g_{m+3} - 3 g_{m+2})^2
// tau8 = (D_m - 2 D_{m+1} + D_{m+2})^2 (Sec. 3, eq:tau8).  The same 13/12 D_j^2 term serves
// the three indicators centred at v_{j+1}.
//
// All indicators are carried scaled by 4 (the exact power-of-two factor only moves the
// exponent): IS' = 4 IS, tau' = 4 tau, with eps' = 4 eps, so every ratio the weights use is
// unchanged.  The caller additionally reconstructs w = 2 f (the split flux without its 1/2),
// which scales IS by 4 again and the flux by 2; the caller passes eps_s = 16 eps and halves
// the flux difference.
//
// Weights (Sec. 3, eq:function and eq:new, normalised as eq:5) are evaluated in the
// algebraically equal single-divide form: with s_k = IS_k + eps, num = IS0 + IS2 - tau5 + eps,
// den = tau5 + eps,
//   alpha_k * den^2 * s0 s1 s2 = c_k * (A num^2 P + tau8 den^2 pi_k) =: c_k B_k,
// P = s0 s1 s2, pi_k = prod_{j != k} s_j,
// and, since sum_k omega_k = 1,
//   fhat = q1 + (c0 B0 (q0 - q1) + c2 B2 (q2 - q1)) / sum_k c_k B_k
// with q0 - q1 = (D_m - D_{m+1})/3, q2 - q1 = (D_{m+1} - D_{m+2})/6 and
// q1 = (v_{m+2} + v_{m+3})/2 - D_{m+1}/6 (eq:4 rewritten with differences).  Numerator and
// denominator are both taken times 10 / c0 (so the linear weights become 1, 6, 3) and every
// B_k times 1/4 (A/4 multiplies num^2 and the fourth difference is not doubled): common
// factors of numerator and denominator that change no weight.
// Every product is >= eps^5 ~ 1e-200 for eps = 1e-40.  The largest, the numerator term
// B2 e_{m+1}, grows as |w|^11: the worst window, an alternating sequence (-w, w, -w, w, -w),
// overflows from |w| ~ 1.1e27 (a step from ~5e27), so window values are limited to
// |w| <= 1e26 (split fluxes of that size).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wzn {

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// 1/x with one v_rcp_f64 and Newton steps; relative error ~1 ulp for normal x.
__device__ __forceinline__ double fast_div(double num, double den) {
  double r = __builtin_amdgcn_rcp(den);
  double e = __builtin_fma(-den, r, 1.0);
  r = __builtin_fma(e, r, r);
  e = __builtin_fma(-den, r, 1.0);
  r = __builtin_fma(e, r, r);
  double q = num * r;
  double res = __builtin_fma(-den, q, num);
  return __builtin_fma(res, r, q);
}

// 1/x with one v_rcp and Newton steps (about 1 ulp for normal x).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(e, r, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(e, r, r);
}
__device__ __forceinline__ float rcp_nr(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  const float e = __builtin_fmaf(-x, r, 1.0f);
  return __builtin_fmaf(e, r, r);
}

// sqrt(x) for x >= 0 from one v_rsq (relative error up to ~5e-8) and one Goldschmidt step:
// with y = rsq(x), s = x y, h = y / 2, s (1 + (1/2 - s h)) has relative error ~1.5 (s h)^2
// deviations (~4e-15).  x = 0 gives 0; x < 0 or NaN gives NaN, as sqrt does.
__device__ __forceinline__ double sqrt_gs(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double s = x * y;
  const double h = 0.5 * y;
  const double r = __builtin_fma(-s, h, 0.5);
  const double t = __builtin_fma(s, r, s);
  return x == 0.0 ? 0.0 : t;
}

// K consecutive WENO-ZN interface values from a window v[0 .. K+3].
// Interface m uses stencil v[m .. m+4] and returns fhat_{m} (the value at the interface
// between v[m+2] and v[m+3]).
// The constant A of eq:function in the form wzn_window<K> takes it: A / 4 for the fp64 window
// (see the normalisation above), A itself for the fp32 window.
template <typename T> __device__ __forceinline__ T window_const(double A);
template <> __device__ __forceinline__ double window_const<double>(double A) { return 0.25 * A; }
template <> __device__ __forceinline__ float window_const<float>(double A) { return float(A); }

// Aq = window_const<double>(A) = A / 4.  Per window element j the shared quantities are the
// differences g_j, D_j, e_j = D_j - D_{j+1} and 13/3 D_j^2 + eps (so that each s_k = IS_k + eps
// is one fma); per interface: tau5 = |s0 - s2|, num = 2 min(s0, s2) - eps (s0 + s2 - |s0 - s2|
// is 2 min(s0, s2), so this is IS0 + IS2 - tau5 + eps up to one rounding; only num^2 enters C),
// b = e_m - e_{m+1}, q1 = v_{m+2} + g_{m+2}/2 - D_{m+1}/6, q0 - q1 = e_m/3, q2 - q1 = e_{m+1}/6.
// The quotient of the nonlinear correction comes from one v_rcp_f64 (relative error up to
// ~5e-8) and one correction folded into the final fma: with r = rcp(S) and e = 1 - S r,
// fhat = q1 + (nr r)(1 + e), whose correction term has relative error ~e^2 (~2e-15).
// WT selects the nonlinear weights: WEIGHTS_ZN, the paper's (Sec. 3, eq:new), or WEIGHTS_Z,
// the WENO-Z weights with q = 1 the paper compares against (Sec. 2.2, eq:15),
// alpha_k = c_k (1 + tau5/(IS_k + eps)).  In the product form above the latter is
// B_k = P + tau5 pi_k (Aq unused), the same normalisation.
enum { WEIGHTS_ZN = 0, WEIGHTS_Z = 1 };

template <int K, int WT = WEIGHTS_ZN>
__device__ __forceinline__ void wzn_window(const double* v, double* fh, double eps_s,
                                           double Aq) {
  constexpr int NG = K + 3;
  constexpr int ND = K + 2;
  double g[NG];
#pragma unroll
  for (int j = 0; j < NG; ++j) g[j] = v[j + 1] - v[j];
  double D[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) D[j] = g[j + 1] - g[j];
  // per-centre 13/3 D^2 + eps (indicators scaled by 4)
  double DD[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) DD[j] = __builtin_fma(D[j] * (13.0 / 3.0), D[j], eps_s);
  double e[K + 1];
#pragma unroll
  for (int j = 0; j <= K; ++j) e[j] = D[j] - D[j + 1];

#pragma unroll
  for (int m = 0; m < K; ++m) {
    // 3 g_{m+1} - g_m = 2 g_{m+1} + D_m and g_{m+3} - 3 g_{m+2} = D_{m+2} - 2 g_{m+2}: inline
    // constants, so no operand has to be copied for an accumulating fma
    const double E0 = __builtin_fma(2.0, g[m + 1], D[m]);
    const double E1 = g[m + 1] + g[m + 2];
    const double E2 = __builtin_fma(-2.0, g[m + 2], D[m + 2]);
    const double s0 = __builtin_fma(E0, E0, DD[m]);
    const double s1 = __builtin_fma(E1, E1, DD[m + 1]);
    const double s2 = __builtin_fma(E2, E2, DD[m + 2]);

    const double t5 = __builtin_fabs(s0 - s2);
    const double p0 = s1 * s2, p1 = s0 * s2, p2 = s0 * s1;
    // B_k = GP + H pi_k
    double GP, H;
    if constexpr (WT == WEIGHTS_Z) {
      GP = s0 * p0;
      H = t5;
    } else {
      const double num = __builtin_fma(2.0, __builtin_fmin(s0, s2), -eps_s);
      const double den = t5 + eps_s;
      // tau8 (in the units of the scaled indicators) = (2 b)^2, b = D_m - 2 D_{m+1} + D_{m+2};
      // H = tau8 den^2 / 4, GP = A num^2 P / 4
      const double b = e[m] - e[m + 1];
      const double bd = b * den;
      H = bd * bd;
      GP = ((Aq * num) * num) * (s0 * p0);
    }
    const double B0 = __builtin_fma(H, p0, GP);
    const double B1 = __builtin_fma(H, p1, GP);
    const double B2 = __builtin_fma(H, p2, GP);
    // numerator and denominator / 6: S = B0/6 + B1 + B2/2 accumulates into B1, which nothing
    // else reads, so no copy of B0 or B2 is needed
    const double S = __builtin_fma(1.0 / 6.0, B0, __builtin_fma(0.5, B2, B1));
    const double x0 = e[m] * (1.0 / 18.0);
    const double x2 = e[m + 1] * (1.0 / 12.0);
    const double nr = __builtin_fma(B0, x0, B2 * x2);
    const double base = __builtin_fma(-1.0 / 6.0, D[m + 1], __builtin_fma(0.5, g[m + 2], v[m + 2]));
    const double r = __builtin_amdgcn_rcp(S);
    const double ope = __builtin_fma(-S, r, 2.0);  // 1 + e
    fh[m] = __builtin_fma(nr * r, ope, base);
  }
}


// ---------------------------------------------------------------------------- fp32 weights
// In fp32 the product form above underflows (eps^5) and the literal form overflows (C and
// tau8/eps reach 1e70), so the weights are evaluated in a scale-safe normalisation of the
// same quantities: dividing every alpha_k by tau8/m with m = min_k s_k,
//   alpha_k ~ c_k (Q + m/s_k),   Q = C m / tau8 = A (num/den)^2 m / tau8,
// where m/s_k lies in (0, 1] and Q is clamped at 1e30 (beyond which the weights equal c_k
// to fp32 precision).  tau8 = 0 gives omega = c exactly.  eps must keep 16 eps normal.
__device__ __forceinline__ float fast_div(float num, float den) {
  return num * __builtin_amdgcn_rcpf(den);
}

template <int K, int WT = WEIGHTS_ZN>
__device__ __forceinline__ void wzn_window(const float* v, float* fh, float eps_s, float A) {
  static_assert(WT == WEIGHTS_ZN, "fp32 runs the paper's weights only");
  constexpr int NG = K + 3;
  constexpr int ND = K + 2;
  float g[NG];
#pragma unroll
  for (int j = 0; j < NG; ++j) g[j] = v[j + 1] - v[j];
  float D[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) D[j] = g[j + 1] - g[j];
  float DD[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) DD[j] = (D[j] * (13.0f / 3.0f)) * D[j];
#pragma unroll
  for (int m = 0; m < K; ++m) {
    const float E0 = __builtin_fmaf(3.0f, g[m + 1], -g[m]);
    const float E1 = g[m + 1] + g[m + 2];
    const float E2 = __builtin_fmaf(-3.0f, g[m + 2], g[m + 3]);
    const float IS0 = __builtin_fmaf(E0, E0, DD[m]);
    const float IS1 = __builtin_fmaf(E1, E1, DD[m + 1]);
    const float IS2 = __builtin_fmaf(E2, E2, DD[m + 2]);
    const float t5 = __builtin_fabsf(IS0 - IS2);
    const float num = ((IS0 + IS2) - t5) + eps_s;
    const float den = t5 + eps_s;
    const float s0 = IS0 + eps_s, s1 = IS1 + eps_s, s2 = IS2 + eps_s;
    const float b = __builtin_fmaf(-2.0f, D[m + 1], D[m] + D[m + 2]);
    const float tau = 4.0f * b * b;  // 4 tau8 in the scaled units
    const float mn = fminf(s0, fminf(s1, s2));
    const float r = fast_div(num, den);
    float Q;
    if (tau > 0.0f) {
      const float mt = fast_div(mn, tau);
      Q = fminf(fminf(A * r, 1e30f) * fminf(r * mt, 1e30f), 1e30f);
    } else {
      Q = 1e30f;
    }
    const float B0 = 0.1f * (Q + fast_div(mn, s0));
    const float B1 = 0.6f * (Q + fast_div(mn, s1));
    const float B2 = 0.3f * (Q + fast_div(mn, s2));
    const float S = B0 + B1 + B2;
    const float x0 = (D[m] - D[m + 1]) * (1.0f / 3.0f);
    const float x2 = (D[m + 1] - D[m + 2]) * (1.0f / 6.0f);
    const float nr = __builtin_fmaf(B0, x0, B2 * x2);
    const float base = __builtin_fmaf(-1.0f / 6.0f, D[m + 1], 0.5f * (v[m + 2] + v[m + 3]));
    fh[m] = base + fast_div(nr, S);
  }
}

// Max of non-negative doubles through their bit patterns (order preserving; a NaN wins).
// The slot only grows, so a plain read that already holds >= v makes the atomic unnecessary;
// a stale read only costs an atomic that was not needed.  This keeps the number of atomics on
// the one address far below the number of workgroups.
__device__ __forceinline__ void atomic_max_pos(unsigned long long* slot, double v) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  const unsigned long long seen = __atomic_load_n(slot, __ATOMIC_RELAXED);
  if (bits > seen) atomicMax(slot, bits);
}

__device__ __forceinline__ double slot_value(const unsigned long long* slot) {
  return __longlong_as_double((long long)(*slot));
}

// v of another lane by a DPP lane move of both 32-bit halves (CTRL as in the DPP encoding),
// every lane written: a lane whose source lane does not exist for CTRL reads 0 (bound_ctrl),
// so no copy of v has to be made first for lanes the move would leave alone.
template <int CTRL>
__device__ __forceinline__ double dpp_move0(double v) {
  const long long b = __double_as_longlong(v);
  const int lo2 = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
  const int hi2 = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi2 << 32) |
                                          (unsigned)lo2));
}

// The value of lane i - 1 in lane i (lane 0 reads 0; its callers replace it): one DPP
// wave_shr:1 lane move per 32-bit half, in place of a shuffle through the LDS crossbar.  All
// 64 lanes must be active.
__device__ __forceinline__ double lane_prev(double v) { return dpp_move0<0x138>(v); }
__device__ __forceinline__ float lane_prev(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}

// Wave-wide max of 64 active lanes holding non-negative values, returned in every lane: DPP
// lane moves (exchange within quads, row half-mirror, row mirror: every lane of a row holds
// the row's max; then the row broadcasts of lane 15 to the next row and of lane 31 to rows 2
// and 3), read back from lane 63.  A lane whose source does not exist takes max(v, 0) = v, so
// the values must be >= 0 (wave speeds and magnitudes).  VALU lane moves instead of the LDS
// crossbar of shuffles (ds_bpermute): six dependent steps of a few cycles rather than of an
// LDS round trip.  max is exact and its order does not matter, so every result is the same
// bits as a shuffle tree's.
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_move0<0xB1>(v));   // quad_perm [1, 0, 3, 2]
  v = fmax(v, dpp_move0<0x4E>(v));   // quad_perm [2, 3, 0, 1]
  v = fmax(v, dpp_move0<0x141>(v));  // row_half_mirror
  v = fmax(v, dpp_move0<0x140>(v));  // row_mirror
  v = fmax(v, dpp_move0<0x142>(v));  // row_bcast:15
  v = fmax(v, dpp_move0<0x143>(v));  // row_bcast:31
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned)lo));
}

// Workgroup maxima of NF per-thread non-negative values into slot[0 .. NF-1] through LDS
// (R: NF * NT doubles that no thread reads any more): every thread writes its NF values, then
// 32 lanes per value each take the max of NT / 32 of them (R[f][j + 32 q], conflict-free) and
// a 32-lane shuffle tree finishes.  Against NF 64-lane trees on every wave this is NF LDS
// writes per thread and one tree on 32 NF threads.  All NT threads must call it.
template <int NT, int NF>
__device__ __forceinline__ void block_max_lds(const double (&s)[NF], double* R,
                                              unsigned long long* slot) {
  static_assert(NT % 32 == 0 && 32 * NF <= NT, "one 32-lane group per value");
  const int tid = threadIdx.x;
  __syncthreads();  // every read of R's previous contents is done
#pragma unroll
  for (int f = 0; f < NF; ++f) R[f * NT + tid] = s[f];
  __syncthreads();
  if (tid < NF * 32) {
    const int f = tid >> 5, j = tid & 31;
    double m = R[f * NT + j];
#pragma unroll
    for (int q = 1; q < NT / 32; ++q) m = fmax(m, R[f * NT + j + 32 * q]);
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if (j == 0) atomic_max_pos(slot + f, m);
  }
}

}  // namespace wzn
