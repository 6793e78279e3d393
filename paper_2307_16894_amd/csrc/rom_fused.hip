// Dispatcher of the fused online solve: argument set-up, the learned warm
// start, the work list of the persistent form, and the per-tile-count launch.
#include <float.h>
#include <string.h>

#include "rom_fused.h"
#include "rom_fused_args.h"

namespace {

// work list of the active points (order irrelevant: the points are independent)
__global__ void k_compact(int P, const int* __restrict__ active, int* __restrict__ list, int* __restrict__ cnt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  if (active && !active[p]) return;
  list[atomicAdd(cnt, 1)] = p;
}

// list length and queue head to zero (a kernel, so the sequence can be captured in a graph)
__global__ void k_zero2(int* __restrict__ c) {
  if (threadIdx.x < 2) c[threadIdx.x] = 0;
}

// Work list and queue counters of rom_step_noalloc: ROM_NOALLOC_MAX_BATCH
// entries, then the two counters at a 256-byte boundary.  Each device holds
// its own copy; host code uses the address looked up per device at set-up,
// never this name.
constexpr int NOALLOC_CNT = (ROM_NOALLOC_MAX_BATCH + 63) / 64 * 64;
static __device__ __align__(256) int scratch[NOALLOC_CNT + 64];

constexpr int NOALLOC_DEVICES = 64;
int* scratch_ptr[NOALLOC_DEVICES];  // device address of scratch per device (null: not looked up)

}  // namespace

// Once per device, with that device current (called by rom_load).
int rom_noalloc_setup(int device) {
  if (device < 0 || device >= NOALLOC_DEVICES) return ROM_EINVAL;
  if (__atomic_load_n(&scratch_ptr[device], __ATOMIC_ACQUIRE)) return ROM_OK;
  int* ptr = nullptr;
  if (hipGetSymbolAddress(reinterpret_cast<void**>(&ptr), HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
    return ROM_EHIP;
  __atomic_store_n(&scratch_ptr[device], ptr, __ATOMIC_RELEASE);  // the same address from any racing caller
  return ROM_OK;
}

int rom_fused_tiles(int n) { return (n + 5 + 15) / 16; }

int rom_fused_setup() {
  int rc = ROM_OK;
  if (rc == ROM_OK) rc = rom_fused_setup_2();
  if (rc == ROM_OK) rc = rom_fused_setup_3();
  if (rc == ROM_OK) rc = rom_fused_setup_4();
  if (rc == ROM_OK) rc = rom_fused_setup_5();
  if (rc == ROM_OK) rc = rom_fused_setup_6();
  if (rc == ROM_OK) rc = rom_fused_setup_7();
  if (rc == ROM_OK) rc = rom_fused_setup_8();
  return rc;
}

// Kernel arguments of a fused or phased step, the wave split, and the
// learned warm start (features and network prediction enqueued on s).
int rom_fused_prepare(rom_model* h, int P, const double* Fbar, void* state, const rom_opts& o, int32_t* st_out,
                      int32_t* it_out, double* res_out, hipStream_t s, FusedArgs& a, int& split) {
  const int T = rom_fused_tiles(h->n);
  if (T < 2 || T > 8 || 16 * T != h->npad) return ROM_EUNSUPPORTED;
  // the point split needs every tile's accumulator in registers: FP64 up to
  // five column tiles, the FP32 accumulators of the reduced forms up to eight
  const bool point_ok = (T <= 5) || (o.contraction != ROM_DT_F64);
  split = o.split;
  if (split < 0) split = point_ok ? 0 : 1;
  if (split != 0 && split != 1) return ROM_EINVAL;
  if (split == 0 && !point_ok) return ROM_EUNSUPPORTED;
  const StateLayout L = rom_state_layout(h, P);
  memset(&a, 0, sizeof(a));
  a.n = h->n;
  a.m = h->m;
  a.max_iter = o.max_iter;
  a.fixed = o.fixed_iters;
  a.commit = o.commit;
  a.max_sub = o.max_substeps;
  a.tol = o.tol;
  a.inv_area = 1.0 / h->cell_area;
  a.mp = h->mp;
  a.mp2 = h->mp2;
  a.phase = h->phase;
  a.Gt = h->Gt;
  a.Gq = h->Gq;
  a.Fbar = Fbar;
  a.rc = field<double>(state, L, F_RC);
  a.rt = field<double>(state, L, F_RT);
  a.hc = field<double>(state, L, F_HC);
  a.ht = field<double>(state, L, F_HT);
  a.tmu = field<double>(state, L, F_TMU);
  a.muok = field<int>(state, L, F_MUOK);
  a.Pbar = field<double>(state, L, F_PBAR);
  a.Abar = field<double>(state, L, F_ABAR);
  a.st_out = st_out;
  a.it_out = it_out;
  a.res_out = res_out;
  a.rg = field<double>(state, L, F_RG);
  a.sub = field<unsigned int>(state, L, F_SUB);
  a.fbc = field<double>(state, L, F_FBC);
  a.zk = field<double>(state, L, F_ZK);
  a.active = o.active;
  if (o.warm_start == ROM_WARM_MLP) {
    int nin = 0, nout = 0;
    rom_mlp_dims(o.mlp, &nin, &nout);
    if (nin != rom_n_features(h) || nout != h->n) return ROM_EINVAL;
    float* X = field<float>(state, L, F_XF);
    float* DR = field<float>(state, L, F_DR);
    int rc = rom_launch_features(h, P, Fbar, state, X, s);
    if (rc != ROM_OK) return rc;
    rc = rom_mlp_predict(o.mlp, P, X, DR, s);
    if (rc != ROM_OK) return rc;
    a.dr = DR;
  }
  return ROM_OK;
}

int rom_fused_launch(int T, const FusedArgs& a, int prec, int split, int grid, int P, hipStream_t s) {
  switch (T) {
    case 2: return rom_fused_launch_2(a, prec, split, grid, P, s);
    case 3: return rom_fused_launch_3(a, prec, split, grid, P, s);
    case 4: return rom_fused_launch_4(a, prec, split, grid, P, s);
    case 5: return rom_fused_launch_5(a, prec, split, grid, P, s);
    case 6: return rom_fused_launch_6(a, prec, split, grid, P, s);
    case 7: return rom_fused_launch_7(a, prec, split, grid, P, s);
    case 8: return rom_fused_launch_8(a, prec, split, grid, P, s);
    default: return ROM_EUNSUPPORTED;
  }
}

int rom_phased_cs(int T, const FusedArgs& a, int prec, int split, int P, hipStream_t s) {
  switch (T) {
    case 2: return rom_phased_cs_2(a, prec, split, P, s);
    case 3: return rom_phased_cs_3(a, prec, split, P, s);
    case 4: return rom_phased_cs_4(a, prec, split, P, s);
    case 5: return rom_phased_cs_5(a, prec, split, P, s);
    default: return ROM_EUNSUPPORTED;
  }
}

// opts.abar_f64 with a reduced-precision contraction: the step defers the
// final commit of its converged points, and FP64 launches then evaluate each
// of them once more at its trial r (from the same committed history and
// Fbar), form Pbar, Abar and K*^-1 C from that FP64 contraction and
// elimination, and commit: the phased kinematics, material and contraction
// kernels over the list of those points where the ROM has them (n <= 75),
// else the FP64 fused kernel over the batch (points not converged return).
bool rom_refines_abar(const rom_opts& o) { return o.abar_f64 && o.contraction != ROM_DT_F64; }

int rom_refine_abar(const rom_model* h, const FusedArgs& a, int split, int P, void* state, hipStream_t s) {
  const int T = rom_fused_tiles(h->n);
  if (h->npad <= ROM_PHASED_NPAD) return rom_refine_abar_phased(h, a, T <= 5 ? split : 1, P, state, s);
  FusedArgs r = a;
  r.refine = 1;
  r.defer = 0;
  r.resume = 0;
  r.max_iter = 1;
  r.fixed = 0;
  r.tol = DBL_MAX;  // the one evaluation stops as converged (a finite ||f||)
  r.max_sub = 0;
  r.dr = nullptr;
  r.list = nullptr;
  r.nlist = nullptr;
  r.counter = nullptr;
  // the FP64 accumulators of the point split fit up to five column tiles
  return rom_fused_launch(T, r, ROM_DT_F64, T <= 5 ? split : 1, 0, P, s);
}

int rom_phased_solve(int T, const FusedArgs& a, int P, hipStream_t s) {
  switch (T) {
    case 2: return rom_phased_solve_2(a, P, s);
    case 3: return rom_phased_solve_3(a, P, s);
    case 4: return rom_phased_solve_4(a, P, s);
    default: return ROM_EUNSUPPORTED;
  }
}

int rom_launch_step_fused(rom_model* h, int P, const double* Fbar, void* state, const rom_opts& o,
                          int32_t* st_out, int32_t* it_out, double* res_out, hipStream_t s) {
  FusedArgs a;
  int split = 0;
  int rc = rom_fused_prepare(h, P, Fbar, state, o, st_out, it_out, res_out, s, a, split);
  if (rc != ROM_OK) return rc;
  int grid = 0;
  if (o.grid_per_cu > 0) {
    const StateLayout L = rom_state_layout(h, P);
    int* cnt = field<int>(state, L, F_COUNT) + 4;
    int* list = field<int>(state, L, F_LIST);
    k_zero2<<<1, 64, 0, s>>>(cnt);
    k_compact<<<(P + 255) / 256, 256, 0, s>>>(P, o.active, list, cnt);
    a.list = list;
    a.nlist = cnt;
    a.counter = cnt + 1;
    grid = o.grid_per_cu * h->ncu;
    if (hipGetLastError() != hipSuccess) return ROM_EHIP;
  }
  const bool refine = rom_refines_abar(o);
  a.defer = refine ? 1 : 0;
  if (rom_timing_mark(h, 0, s) != ROM_OK) return ROM_EHIP;
  rc = rom_fused_launch(rom_fused_tiles(h->n), a, o.contraction, split, grid, P, s);
  if (rc == ROM_OK && refine) rc = rom_refine_abar(h, a, split, P, state, s);
  if (rom_timing_mark(h, 1, s) != ROM_OK) return ROM_EHIP;
  return rc;
}

// The fused form on a persistent grid with its work list and counters in the
// device's static scratch: no allocation, no timing marks (they create events).
int rom_launch_step_noalloc(rom_model* h, int P, const double* Fbar, void* state, const rom_opts& o,
                            int32_t* st_out, int32_t* it_out, double* res_out, hipStream_t s) {
  if (P > ROM_NOALLOC_MAX_BATCH) return ROM_ESCRATCH;
  if (h->device < 0 || h->device >= NOALLOC_DEVICES) return ROM_EHIP;
  int* base = __atomic_load_n(&scratch_ptr[h->device], __ATOMIC_ACQUIRE);
  if (!base) return ROM_EHIP;  // rom_load looks it up; a handle without it was not loaded here
  FusedArgs a;
  int split = 0;
  int rc = rom_fused_prepare(h, P, Fbar, state, o, st_out, it_out, res_out, s, a, split);
  if (rc != ROM_OK) return rc;
  int* list = base;
  int* cnt = base + NOALLOC_CNT;
  k_zero2<<<1, 64, 0, s>>>(cnt);  // the last call's counters: cleared by a kernel, as in a captured graph
  k_compact<<<(P + 255) / 256, 256, 0, s>>>(P, o.active, list, cnt);
  if (hipGetLastError() != hipSuccess) return ROM_EHIP;
  a.list = list;
  a.nlist = cnt;
  a.counter = cnt + 1;
  const int grid = (o.grid_per_cu > 0 ? o.grid_per_cu : 2) * h->ncu;
  const bool refine = rom_refines_abar(o);
  a.defer = refine ? 1 : 0;
  rc = rom_fused_launch(rom_fused_tiles(h->n), a, o.contraction, split, grid, P, s);
  if (rc == ROM_OK && refine) rc = rom_refine_abar(h, a, split, P, state, s);  // work lists in the state: no scratch
  return rc;
}
