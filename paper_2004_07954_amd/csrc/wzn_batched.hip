// Persistent batched TVD-RK3 run of many independent 1D Euler problems of uneven length.
//
// One launch advances every instance by nsteps steps.  Workgroups pull instance indices from
// a device work-queue counter (in the caller's processing order, e.g. longest first) and
// advance their instance through all 3 * nsteps stages, tile by tile, with the same row tile
// as the one-instance path (wzn_tile.hpp).  Stages of one instance are separated by workgroup
// barriers, so the global Lax-Friedrichs alpha of each stage and the dt of each step
// (dt = cfl dx_i / max(|u| + c) of the instance's U^n, Sec. 4.3) are workgroup reductions:
// no grid-wide synchronisation and no atomics except the queue counter.  Every workgroup
// leaves the loop once the counter passes the batch size.
#include <hip/hip_runtime.h>

#include "wzn_device.hpp"
#include "wzn_host.hpp"
#include "wzn_rows.hpp"
#include "wzn_tile.hpp"

namespace wzn {

struct BatchArgs {
  double* u;                // [3][total] concatenated instances (in/out)
  double* U1;               // [3][total] stage scratch
  double* U2;               // [3][total] stage scratch
  const int64_t* offsets;   // [batch + 1]
  const double* dx;         // [batch]
  const int32_t* order;     // [batch] processing order, or null (0 .. batch-1)
  int32_t batch;
  int32_t nsteps;
  int64_t total;
  double cfl, gamma, eps_s, A;
  int bc;
  unsigned long long* counter;
  double* dt_out;           // [batch][nsteps] or null
};

template <int NT, int K, bool SPLIT>
__global__ __launch_bounds__(NT) void batched_kernel(BatchArgs b) {
  constexpr int TT = NT * K;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* W = reinterpret_cast<double*>(lds_raw);
  __shared__ double EX[tile_ex_elems<SYS_EULER1, NT>()];
  __shared__ double red[NT / 64];
  __shared__ int next;
  const int tid = threadIdx.x;

  for (;;) {
    if (tid == 0) next = (int)atomicAdd(b.counter, 1ull);
    __syncthreads();
    const int qi = next;
    __syncthreads();  // every thread has read `next` before it is overwritten
    if (qi >= b.batch) break;
    const int inst = b.order ? b.order[qi] : qi;
    if (inst < 0 || inst >= b.batch) continue;  // an order entry out of range: skipped
    const int64_t off = b.offsets[inst];
    const int64_t n = b.offsets[inst + 1] - off;
    // malformed instance (or one longer than a row may be): left untouched
    if (n < 6 || n > ((int64_t)1 << 30) || off < 0 || off + n > b.total) continue;
    const double dx = b.dx[inst];

    RowArgs<double> a{};
    a.n = n;
    a.plane = b.total;
    a.row_stride = 0;
    a.dx = dx;
    a.bc = b.bc;
    a.mode = MODE_STAGE;
    a.gamma = b.gamma;
    a.eps_s = b.eps_s;
    a.A = b.A;

    // max |u| + c of the instance's initial state
    double smax = 0.0;
    for (int64_t i = tid; i < n; i += NT) {
      const double U[3] = {b.u[off + i], b.u[b.total + off + i], b.u[2 * b.total + off + i]};
      smax = fmax(smax, wave_speed_1d<SYS_EULER1>(U, 0.0, b.gamma));
    }
    double alpha = block_max<NT>(smax, red);
    const int64_t ntiles = (n + TT - 1) / TT;
    for (int step = 0; step < b.nsteps; ++step) {
      const double dt = b.cfl * dx / alpha;  // alpha here is max(|u| + c) of U^n
      if (b.dt_out && tid == 0) b.dt_out[(int64_t)inst * b.nsteps + step] = dt;
      for (int k = 0; k < 3; ++k) {
        a.uin = k == 0 ? b.u : (k == 1 ? b.U1 : b.U2);
        a.out = k == 0 ? b.U1 : (k == 1 ? b.U2 : b.u);
        a.un = k == 0 ? nullptr : b.u;
        a.rk_a = k == 0 ? 0.0 : (k == 1 ? 3.0 / 4.0 : 1.0 / 3.0);
        a.rk_b = k == 0 ? 1.0 : (k == 1 ? 1.0 / 4.0 : 2.0 / 3.0);
        smax = 0.0;
        for (int64_t t = 0; t < ntiles; ++t)
          row_tile<NT, K, SYS_EULER1, double, true, SPLIT>(a, t * TT, off, alpha, dt, W, EX, smax);
        alpha = block_max<NT>(smax, red);  // alpha of the next stage's input
      }
    }
  }
}

template <int NT, int K, bool SPLIT>
static int launch_batched_t(const BatchArgs& b, int blocks_per_cu, hipStream_t s) {
  const size_t lds = tile_lds_bytes<NT, K, SYS_EULER1, double, SPLIT>();
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute((const void*)batched_kernel<NT, K, SPLIT>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return set_error(WZN_ERR_HIP, "hipFuncSetAttribute(batched_kernel) failed");
    attr_set = true;
  }
  int dev = 0, cus = 0, occ = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return set_error(WZN_ERR_HIP, "cannot query the device");
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)batched_kernel<NT, K, SPLIT>, NT,
                                                   lds) != hipSuccess || occ < 1)
    occ = 1;
  int per_cu = blocks_per_cu > 0 ? (blocks_per_cu < occ ? blocks_per_cu : occ) : occ;
  int64_t grid = (int64_t)cus * per_cu;
  if (grid > b.batch) grid = b.batch;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((batched_kernel<NT, K, SPLIT>), dim3((unsigned)grid), dim3(NT), lds, s, b);
  return check_launch("batched_kernel");
}

int batched_rk3_run_1d(const wzn_params* p, double* u, double* stage, int64_t total,
                       const int64_t* offsets, const double* dx, const int32_t* order,
                       int32_t batch, int32_t nsteps, double cfl, const wzn_batch_tuning* tn,
                       double* dt_out, Workspace* ws, hipStream_t s) {
  BatchArgs b{};
  b.u = u;
  b.U1 = stage;
  b.U2 = stage + 3 * total;
  b.offsets = offsets;
  b.dx = dx;
  b.order = order;
  b.batch = batch;
  b.nsteps = nsteps;
  b.total = total;
  b.cfl = cfl;
  b.gamma = p->gamma;
  b.eps_s = 16.0 * p->eps;
  b.A = p->A;
  b.bc = p->bc_x;
  b.counter = ws->counter;
  b.dt_out = dt_out;
  int st = launch_zero_words(ws->counter, 1, s);
  if (st) return st;
  const int nt = tn ? tn->nt : 128, k = tn ? tn->k : 2, bpc = tn ? tn->blocks_per_cu : 0;
  const int lay = tn ? tn->layout : ROW_LDS_TILE;
  if (lay == ROW_LDS_TILE) {
    if (nt == 64 && k == 4) return launch_batched_t<64, 4, false>(b, bpc, s);
    if (nt == 64 && k == 2) return launch_batched_t<64, 2, false>(b, bpc, s);
    if (nt == 128 && k == 2) return launch_batched_t<128, 2, false>(b, bpc, s);
    if (nt == 128 && k == 4) return launch_batched_t<128, 4, false>(b, bpc, s);
    if (nt == 256 && k == 1) return launch_batched_t<256, 1, false>(b, bpc, s);
    if (nt == 256 && k == 2) return launch_batched_t<256, 2, false>(b, bpc, s);
    if (nt == 256 && k == 4) return launch_batched_t<256, 4, false>(b, bpc, s);
  } else if (lay == ROW_LDS_SPLIT) {
    if (nt == 128 && k == 4) return launch_batched_t<128, 4, true>(b, bpc, s);
    if (nt == 256 && k == 2) return launch_batched_t<256, 2, true>(b, bpc, s);
    if (nt == 256 && k == 4) return launch_batched_t<256, 4, true>(b, bpc, s);
  }
  return set_error(WZN_ERR_ARG, "unsupported batched tuning (nt=%d, k=%d, layout=%d)", nt, k,
                   lay);
}

}  // namespace wzn
