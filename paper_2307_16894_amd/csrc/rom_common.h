// Shared definitions of the ROM library: the loaded model, the state layout
// and small device helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/podecm.h"
#include "j2_device.h"

#define ROM_NMAX 128       // largest supported number of modes n
#define ROM_REC_ROWS 20    // phased-form ECM-point record: D (16, FP32 pairs in 8 in the BF16 form), P (4)
#define ROM_PHASED_NPAD 80  // widest contraction tile set of the phased form (n <= 75)
#define ROM_ALIGN 256

// Loaded ROM (Algorithm 1, offline output) resident on one device.
struct rom_model {
  int device;
  int n, m, c, kind, n_mu;
  int npad;              // padded width of the contraction tiles
  int ncu;               // compute units of the device
  double E, nu, sy0, H, r0, void_area, cell_area;
  J2Params mp;
  J2Params mp2;  // second phase (two-phase cells)
  int* phase;    // [m] phase of every ECM point (0: mp, 1: mp2), null for a single-phase cell
  double* w;    // [m] ECM weights
  double* Gt;   // [n][4][m] mode gradients, point fastest (per-lane kinematics)
  double* Gq;   // [m][4][npad] mode gradients, mode fastest, zero padded (contractions)
  double* Gd;   // [c][4][m] transformation-mode gradients, point fastest
  float* Gq32;  // [m][4][npad] FP32 copy of Gq
  uint16_t* Gq16;  // [m][4][npad] BF16 copy of Gq
  // phased form: side stream of the fused kernel that finishes the slow
  // points while the phased evaluations go on (created at first use)
  hipStream_t aux;
  hipEvent_t ev_fork, ev_join;
  // kernel timing (measurement support)
  int timing;
  int nev;                 // event pairs recorded since enable
  int cap;                 // event pairs allocated
  hipEvent_t* ev;          // [2 * cap]
};

// Material of ECM point q: the second phase where the cell has one and the
// point lies in it.  By value: a reference into a kernel's argument struct
// would make the compiler copy the whole struct to private memory.
__host__ __device__ inline J2Params point_params(J2Params mp, J2Params mp2, const int* phase, int q) {
  const bool two = phase && phase[q];
  J2Params r;
  r.G = two ? mp2.G : mp.G;
  r.lam = two ? mp2.lam : mp.lam;
  r.K = two ? mp2.K : mp.K;
  r.sy0 = two ? mp2.sy0 : mp.sy0;
  r.H = two ? mp2.H : mp.H;
  return r;
}

// Bit of the sub-step record (ROM_FIELD_SUBSTEPS) for a converged sub-step
// ending at t_done / 2^D of the load step: exact on the 1/32 grid up to
// D = 5, the 1/32 cell holding the end point beyond.
__host__ __device__ inline unsigned int substep_bit(int t_done, int D) {
  const int k = (D <= 5) ? (t_done << (5 - D)) - 1 : (t_done - 1) >> (D - 5);
  return 1u << k;
}

// Record the start / stop event of a timed launch; no-ops unless enabled.
int rom_timing_mark(rom_model* h, int stop, hipStream_t s);

// warm-start network entry points used by rom_step (mlp.hip)
int rom_mlp_predict(struct rom_mlp* m, int B, const float* X, float* Y, hipStream_t s);
int rom_mlp_dims(const struct rom_mlp* m, int* n_in, int* n_out);
int rom_launch_features(const rom_model* h, int P, const double* Fbar, const void* state, float* X, hipStream_t s);

// Internal state fields (public ones first, same numbering as ROM_FIELD_*).
enum {
  F_RC = 0, F_RT, F_HC, F_HT, F_TMU, F_PBAR, F_ABAR, F_MUOK, F_FBC, F_RG, F_SUB,
  F_DONE, F_STATUS, F_ITERS, F_RES, F_COUNT, F_XF, F_DR, F_MU, F_LIST,
  F_D, F_W, F_K, F_F, F_PIV,
  F_REC, F_PHI, F_PHD, F_LIST2, F_LIST3, F_LIST4, F_HKIN, F_ZK, F_SYS,
  F_NFIELDS
};

// Phased form up to ROM_SOLVE_NPAD columns: the system [K | f | C] of each
// point (npad columns of n rows) with the effective-quantity rows and ||f||
// (24 doubles), handed from the contraction launch to the solve launch.
#define ROM_SOLVE_NPAD 64
__host__ __device__ inline size_t rom_sys_stride(int npad, int n) { return (size_t)npad * n + 24; }

// per-point inputs of the warm-start network: mu, Fbar - Fbar_committed, r, 8 statistics
static inline int rom_n_features(const rom_model* h) { return h->n_mu + 4 + h->n + 8; }

struct StateLayout {
  size_t off[F_NFIELDS];
  size_t total;
};

static inline size_t rom_align_up(size_t x) { return (x + ROM_ALIGN - 1) / ROM_ALIGN * ROM_ALIGN; }

static inline StateLayout rom_state_layout(const rom_model* h, size_t P) {
  const size_t n = h->n, m = h->m;
  size_t sz[F_NFIELDS];
  sz[F_RC] = P * n * 8;
  sz[F_RT] = P * n * 8;
  sz[F_HC] = P * 6 * m * 8;
  sz[F_HT] = P * 6 * m * 8;
  sz[F_TMU] = P * 5 * m * 8;
  sz[F_PBAR] = P * 4 * 8;
  sz[F_ABAR] = P * 16 * 8;
  sz[F_MUOK] = P * 4;
  sz[F_FBC] = P * 4 * 8;
  sz[F_RG] = P * n * 8;
  sz[F_SUB] = P * 4;
  sz[F_DONE] = P * 4;
  sz[F_STATUS] = P * 4;
  sz[F_ITERS] = P * 4;
  sz[F_RES] = P * 8;
  sz[F_COUNT] = 64;
  sz[F_XF] = P * (size_t)rom_n_features(h) * 4;
  sz[F_DR] = P * n * 4;
  sz[F_MU] = P * (size_t)h->n_mu * 8;
  sz[F_LIST] = P * 4;
  sz[F_D] = P * 16 * m * 8;
  sz[F_W] = P * 4 * m * 8;
  sz[F_K] = P * n * n * 8;
  sz[F_F] = P * n * 8;
  sz[F_PIV] = P * n * 4;
  // phased form: per-point records between the material and contraction launches
  sz[F_REC] = (h->npad <= ROM_PHASED_NPAD) ? P * m * ROM_REC_ROWS * 8 : 0;
  sz[F_PHI] = P * 2 * 4;
  sz[F_PHD] = P * 2 * 8;
  sz[F_LIST2] = P * 4;
  sz[F_LIST3] = P * 4;
  sz[F_LIST4] = P * 4;
  sz[F_HKIN] = (h->npad <= ROM_PHASED_NPAD) ? P * 4 * m * 8 : 0;
  sz[F_ZK] = P * n * 4 * 8;  // K*^-1 C at the returned state (shape sensitivities)
  sz[F_SYS] = (h->npad <= ROM_SOLVE_NPAD) ? P * rom_sys_stride(h->npad, (int)n) * 8 : 0;
  StateLayout L;
  size_t o = 0;
  for (int i = 0; i < F_NFIELDS; ++i) {
    L.off[i] = o;
    o += rom_align_up(sz[i]);
  }
  L.total = o;
  return L;
}

template <typename T>
static inline T* field(void* base, const StateLayout& L, int f) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + L.off[f]);
}
