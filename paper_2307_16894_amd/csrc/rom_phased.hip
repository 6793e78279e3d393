// Phased form of the online solve.  The first evaluations of the Newton
// iteration (eq. red_newton) of every point of the batch run as three
// launches each:
//   kinematics:  H = sum_i r_i G_i(q) of every listed point as one FP64
//                MFMA product (the mode gradients read once for all points);
//   material:    one lane per ECM point of every listed point (return map,
//                tangent and the contraction record of Appendix A and eqs.
//                forcevector_ecm / stiffnessmatrix_ecm), the lanes packed
//                across points;
//   contraction: one workgroup per listed point (the MFMA contraction of the
//                records, then, up to 64 columns, the system to HBM; wider,
//                the elimination, status and Newton update in place), a
//                kernel with a register budget of its own;
//   solve:       up to 64 columns, one wave per listed point (the
//                elimination with the row of the lane in registers, the
//                status, the Newton update or the effective quantities), no
//                workgroup barrier.
// After ph_k evaluations the points still running (and any attempt that
// failed with load-step cutting on) are finished by the fused kernel as a
// persistent grid, which resumes each point from the state left here.  Points
// that converge slowly at evaluation ph_early (likely to fail the plain step
// and be cut into sub-steps, a long chain of evaluations) are handed over
// then, to a fused kernel on a side stream that runs beside the remaining
// phased evaluations.  Where a point's evaluations run does not change them:
// the results are the same bit for bit.  The list lengths stay on the device:
// nothing is read back.  The step is launched eagerly (not inside a graph
// capture, which it refuses).
#include <string.h>

#include "rom_fused.h"
#include "rom_fused_impl.h"

namespace {

// phased evaluations (default; with the learned warm start, which needs
// fewer evaluations per point, PH_EVALS_WARM and no early hand-over: measured
// faster on the n = 40 workload, 1.72 -> 1.67 ms per BF16 step)
constexpr int PH_EVALS = 6, PH_EVALS_WARM = 4;
// early hand-over (default): after this many evaluations, points whose ||f||
// fell by less than the factor PH_SLOW in the last update
constexpr int PH_EARLY = 3;
constexpr double PH_SLOW = 0.3;
constexpr int PH_EARLY_GRID = 1;  // workgroups per compute unit of the side-stream fused kernel

__global__ void k_zero6(int* __restrict__ c) {
  if (threadIdx.x < 6) c[threadIdx.x] = 0;
}

// initial guess (committed r plus the predicted increment), the evaluation
// state, and the list of the points taking part
__global__ void k_ph_begin(const FusedArgs a, int P) {
  const int n = a.n;
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long long)P * n) return;
  const int p = (int)(g / n), i = (int)(g - (long long)p * n);
  if (a.active && !a.active[p]) return;
  if (!a.muok[p]) {
    if (i == 0)
      for (int k = 0; k < 16; ++k) bad_mu_outputs(a, p, k);
    return;
  }
  double v = a.rc[(size_t)p * n + i];
  if (a.dr) v += (double)a.dr[(size_t)p * n + i];
  a.rg[(size_t)p * n + i] = v;
  a.rt[(size_t)p * n + i] = v;
  if (i == 0) {
    a.phi[2 * (size_t)p] = 0;
    a.phi[2 * (size_t)p + 1] = 0;
    a.lout[atomicAdd(a.cout, 1)] = p;
  }
}

// Kinematics launch: H = G R for the listed points as an FP64 MFMA product,
// rows (b, q) of the mode gradients (Gt, [n][4][m]) against the trial r of
// each listed point, four modes per instruction in mode order.  The FP64
// instruction adds its four products to the accumulator as a chain of fma
// in that order, so each H entry is the same fma chain over the modes as the
// fused kernel's per-lane kinematics (zero modes past n add nothing).
// Workgroup: 64 rows (a wave each 16) by 64 list entries (four 16-column
// tiles per wave).
__global__ __launch_bounds__(256) void k_ph_kin(const FusedArgs a) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = a.n, m = a.m, rows = 4 * m;
  const int cnt = *a.cin;
  const int j0 = blockIdx.y * 64;
  if (j0 >= cnt) return;
  const int r0 = blockIdx.x * 64 + wave * 16;
  if (r0 >= rows) return;
  const int li = lane & 15, lk = lane >> 4;
  const int ra = min(r0 + li, rows - 1);  // A row of this lane (rows past the end repeat the last; not stored)
  int pj[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int j = j0 + 16 * t + li;
    pj[t] = (j < cnt) ? a.lin[j] : -1;
  }
  d4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = (d4){0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < n; s += 4) {
    const int i = s + lk;
    const double av = (i < n) ? a.Gt[(size_t)i * rows + ra] : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double bv = (i < n && pj[t] >= 0) ? a.rt[(size_t)pj[t] * n + i] : 0.0;
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
    }
  }
  // output: register jj of lane l is row (l >> 4) + 4 jj, column l & 15
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int j = j0 + 16 * t + li;
    if (j >= cnt) continue;
    double* Hj = a.hkin + (size_t)j * rows;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int r = r0 + lk + 4 * jj;
      if (r < rows) Hj[r] = acc[t][jj];
    }
  }
}

// Material launch: lane g of the grid takes ECM point g mod m of list entry
// g / m: F from the kinematics launch's H, the return map, and the record.
// Block 0 also clears the count of the list the following contraction
// launch fills.
template <int PREC>
__global__ __launch_bounds__(256) void k_ph_mat(const FusedArgs a) {
  const int tid = threadIdx.x, m = a.m;
  if (blockIdx.x == 0 && tid == 0) *a.cout = 0;
  const long long cnt = *a.cin;
  const long long g = (long long)blockIdx.x * 256 + tid;
  if (g >= cnt * m) return;
  const int idx = (int)(g / m), q = (int)(g - (long long)idx * m), p = a.lin[idx];
  const double Fb[4] = {a.Fbar[4 * (size_t)p], a.Fbar[4 * (size_t)p + 1], a.Fbar[4 * (size_t)p + 2],
                        a.Fbar[4 * (size_t)p + 3]};
  double* rec = a.rec + (size_t)p * ROM_REC_ROWS * m + q;
  const double* tmu = a.tmu + (size_t)p * 5 * m;
  const double* H = a.hkin + (size_t)idx * 4 * m + q;
  double F[4], D[16], P[4], Fi[4], wJ;
#pragma unroll
  for (int k = 0; k < 4; ++k) Fi[k] = tmu[k * m + q];
  kin_F(Fb, H[0], H[m], H[2 * m], H[3 * m], Fi, F);
  point_material(F, m, q, tmu, a.hc + (size_t)p * 6 * m, a.ht + (size_t)p * 6 * m, point_params(a.mp, a.mp2, a.phase, q),
                 D, P, Fi, wJ);
  put_record_d<PREC>(rec, m, D);
#pragma unroll
  for (int k = 0; k < 4; ++k) rec[(size_t)(rec_p_row<PREC>() + k) * m] = P[k];
}

int launch_mat(const FusedArgs& a, int prec, int P, int m, hipStream_t s) {
  k_ph_kin<<<dim3((unsigned int)((4 * m + 63) / 64), (unsigned int)((P + 63) / 64)), 256, 0, s>>>(a);
  const unsigned int blocks = (unsigned int)(((long long)P * m + 255) / 256);
  if (prec == ROM_DT_F64)
    k_ph_mat<PREC_F64><<<blocks, 256, 0, s>>>(a);
  else if (prec == ROM_DT_F32)
    k_ph_mat<PREC_F32><<<blocks, 256, 0, s>>>(a);
  else
    k_ph_mat<PREC_BF16><<<blocks, 256, 0, s>>>(a);
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

// the points a step reported converged (the refining launches of abar_f64)
__global__ void k_list_converged(int P, const int* __restrict__ st, const int* __restrict__ active,
                                 int* __restrict__ list, int* __restrict__ cnt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  if (active && !active[p]) return;
  const int v = st[p];
  if (v == ROM_ST_CONVERGED || v == ROM_ST_FALLBACK) list[atomicAdd(cnt, 1)] = p;
}

}  // namespace

// abar_f64 after a reduced-precision step, as phased launches: the converged
// points listed, then one FP64 kinematics, material and contraction launch
// over them (the contraction kernel's refining branch eliminates, writes the
// effective quantities and commits).
int rom_refine_abar_phased(const rom_model* h, const FusedArgs& a, int split, int P, void* state, hipStream_t s) {
  const StateLayout L = rom_state_layout(h, P);
  int* cnt = field<int>(state, L, F_COUNT) + 8;
  int* list = field<int>(state, L, F_LIST);
  FusedArgs b = a;
  b.refine = 1;
  b.defer = 0;
  b.resume = 0;
  b.dr = nullptr;
  b.rec = field<double>(state, L, F_REC);
  b.hkin = field<double>(state, L, F_HKIN);
  b.phi = field<int>(state, L, F_PHI);
  b.phd = field<double>(state, L, F_PHD);
  b.lin = list;
  b.cin = cnt;
  b.sys = nullptr;  // the refining contraction eliminates in place
  // the material kernel clears the count of the list a contraction launch
  // fills next: give it the second list's slot (the refining contraction
  // lists nothing)
  b.lout = field<int>(state, L, F_LIST2);
  b.cout = cnt + 1;
  k_zero6<<<1, 64, 0, s>>>(cnt);
  k_list_converged<<<(P + 255) / 256, 256, 0, s>>>(P, a.st_out, a.active, list, cnt);
  if (hipGetLastError() != hipSuccess) return ROM_EHIP;
  const int rc = launch_mat(b, ROM_DT_F64, P, h->m, s);
  return rc == ROM_OK ? rom_phased_cs(rom_fused_tiles(h->n), b, ROM_DT_F64, split, P, s) : rc;
}

int rom_launch_step_phased(rom_model* h, int P, const double* Fbar, void* state, const rom_opts& o,
                           int32_t* st_out, int32_t* it_out, double* res_out, hipStream_t s) {
  if (h->npad > ROM_PHASED_NPAD) return ROM_EUNSUPPORTED;
  // eager launches only: a graph capture of the step with its side-stream fork
  // and join has crashed the runtime's end of capture (host side), so the
  // phased form refuses capture
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess) return ROM_EHIP;
  if (cap != hipStreamCaptureStatusNone) return ROM_EUNSUPPORTED;
  if ((long long)P * h->m > (1LL << 31) - 256) return ROM_EUNSUPPORTED;
  const bool warm = o.warm_start == ROM_WARM_MLP;
  const int kph = min(o.phased_evals > 0 ? o.phased_evals : (warm ? PH_EVALS_WARM : PH_EVALS), o.max_iter);
  if (kph < 1) return rom_launch_step_fused(h, P, Fbar, state, o, st_out, it_out, res_out, s);
  FusedArgs a;
  int split = 0;
  int rc = rom_fused_prepare(h, P, Fbar, state, o, st_out, it_out, res_out, s, a, split);
  if (rc != ROM_OK) return rc;
  const StateLayout L = rom_state_layout(h, P);
  // counts of list A, list B, the hand-over list, its queue head, the early list, its queue head
  int* cnt = field<int>(state, L, F_COUNT) + 8;
  int* listA = field<int>(state, L, F_LIST);
  int* listB = field<int>(state, L, F_LIST2);
  int* hand = field<int>(state, L, F_LIST3);
  int* early = field<int>(state, L, F_LIST4);
  a.ph_k = kph;
  const int ke = o.phased_early == 0 ? (warm ? -1 : PH_EARLY) : o.phased_early;
  a.ph_early = (ke > 1 && ke < kph) ? ke : 0;
  a.ph_slow = PH_SLOW;
  a.early = early;
  a.cearly = cnt + 4;
  a.rec = field<double>(state, L, F_REC);
  a.hkin = field<double>(state, L, F_HKIN);
  a.phi = field<int>(state, L, F_PHI);
  a.phd = field<double>(state, L, F_PHD);
  a.hand = hand;
  a.chand = cnt + 2;
  // up to ROM_SOLVE_NPAD columns the elimination runs in a launch of its own
  a.sys = (h->npad <= ROM_SOLVE_NPAD) ? field<double>(state, L, F_SYS) : nullptr;
  const int T = rom_fused_tiles(h->n);
  const bool refine = rom_refines_abar(o);
  a.defer = refine ? 1 : 0;
  if (rom_timing_mark(h, 0, s) != ROM_OK) return ROM_EHIP;
  // from here every exit goes through the join and the stop mark below
  k_zero6<<<1, 64, 0, s>>>(cnt);
  {
    FusedArgs b = a;
    b.lout = listA;
    b.cout = cnt;
    k_ph_begin<<<(unsigned int)(((long long)P * h->n + 255) / 256), 256, 0, s>>>(b, P);
  }
  if (hipGetLastError() != hipSuccess) rc = ROM_EHIP;
  bool forked = false;
  for (int e = 0; e < kph && rc == ROM_OK; ++e) {
    FusedArgs b = a;
    b.lin = (e & 1) ? listB : listA;
    b.cin = cnt + (e & 1);
    b.lout = (e & 1) ? listA : listB;
    b.cout = cnt + 1 - (e & 1);
    rc = launch_mat(b, o.contraction, P, h->m, s);
    if (rc == ROM_OK) rc = rom_phased_cs(T, b, o.contraction, split, P, s);
    if (rc == ROM_OK && b.sys) rc = rom_phased_solve(T, b, P, s);
    if (rc == ROM_OK && a.ph_early > 0 && e + 1 == a.ph_early) {
      // fork: the early list to the fused kernel on the side stream
      if (hipEventRecord(h->ev_fork, s) != hipSuccess) {
        rc = ROM_EHIP;
        break;
      }
      if (hipStreamWaitEvent(h->aux, h->ev_fork, 0) != hipSuccess) {
        rc = ROM_EHIP;
        break;
      }
      forked = true;
      FusedArgs f = a;
      f.resume = 1;
      f.list = early;
      f.nlist = cnt + 4;
      f.counter = cnt + 5;
      rc = rom_fused_launch(T, f, o.contraction, split, PH_EARLY_GRID * h->ncu, P, h->aux);
    }
  }
  if (rc == ROM_OK) {
    FusedArgs f = a;
    f.resume = 1;
    f.list = hand;
    f.nlist = cnt + 2;
    f.counter = cnt + 3;
    const int grid = (o.grid_per_cu > 0 ? o.grid_per_cu : 2) * h->ncu;
    rc = rom_fused_launch(T, f, o.contraction, split, grid, P, s);
  }
  // join: the step ends when the side stream's work is done too (also after
  // a failed launch, so that nothing of this step is left running beside s)
  if (forked) {
    const bool joined = hipEventRecord(h->ev_join, h->aux) == hipSuccess &&
                        hipStreamWaitEvent(s, h->ev_join, 0) == hipSuccess;
    if (!joined) {
      (void)hipStreamSynchronize(h->aux);  // the event pair failed: wait on the host instead
      if (rc == ROM_OK) rc = ROM_EHIP;
    }
  }
  if (rc == ROM_OK && refine) rc = rom_refine_abar(h, a, split, P, state, s);
  if (rom_timing_mark(h, 1, s) != ROM_OK && rc == ROM_OK) rc = ROM_EHIP;
  return rc;
}
