// Kernel arguments of the fused online solve (shared by the per-tile-count
// translation units and the dispatcher).
#pragma once
#include "rom_common.h"

struct FusedArgs {
  int n, m, max_iter, fixed, commit;
  int max_sub;  // load-step cutting depth (0: plain step)
  double tol, inv_area;
  J2Params mp;
  J2Params mp2;       // second phase of a two-phase cell
  const int* phase;   // [m] phase of every ECM point, or null
  const double* Gt;
  const double* Gq;
  const double* Fbar;
  double* rc;
  double* rt;
  double* hc;
  double* ht;
  const double* tmu;
  const int* muok;
  double* Pbar;
  double* Abar;
  int* st_out;
  int* it_out;
  double* res_out;
  const int* active;  // active points (NULL: all)
  const int* list;   // work list (queue mode)
  const int* nlist;  // its length (device)
  int* counter;      // next list entry to take (device)
  const float* dr;   // warm-start increments [P][n] (NULL: plain guess)
  double* rg;        // initial guess actually used [P][n]
  unsigned int* sub;  // converged sub-steps of the step, substep_bit() per sub-step [P]
  double* fbc;       // committed Fbar [P][4]
  double* zk;        // K*^-1 C at the returned state [P][n][4]
  // phased form: the first evaluations of attempt 0 as a material launch and a
  // contraction launch per evaluation, the points still running after them
  // handed to the fused kernel, which resumes them from this state
  int ph_k;          // evaluations made by the phased launches
  double* rec;       // ECM-point records [P][ROM_REC_ROWS][m] (point fastest)
  double* hkin;      // H = sum_i r_i G_i(q) of the listed points [list entry][4][m]
  int* phi;          // per point: evaluations made, fell back to the plain guess [P][2]
  double* phd;       // per point: ||f|| of the first and of the latest evaluation [P][2]
  const int* lin;    // points of this evaluation
  const int* cin;    // their count (device)
  int* lout;         // points making the next phased evaluation
  int* cout;         // their count (device)
  int* hand;         // points handed to the fused kernel
  int* chand;        // their count (device)
  int ph_early;      // evaluations after which slow points go to the early list (0: none)
  double ph_slow;    // slow: ||f|| above this fraction of the previous evaluation's
  int* early;        // points handed to the fused kernel on the side stream
  int* cearly;       // their count (device)
  int resume;        // fused kernel: start each point from phi / phd (evaluation phi[0] of attempt 0)
  double* sys;       // phased form up to ROM_SOLVE_NPAD columns: the contraction launch leaves the system of
                     // each point here [P][rom_sys_stride] and a solve launch eliminates (NULL: in place)
  int defer;         // converged points leave their final commit to a refining launch
  int refine;        // fused kernel: one evaluation at the trial r of each point the step reported converged,
                     // its effective quantities, and the commit (statuses, counts and norms kept)
};

// per tile-count entry points (rom_fused_t<T>.hip): launch with the given
// contraction precision, wave split (0 points, 1 tiles), and persistent grid
// (grid > 0: that many workgroups pulling from the work list in the args;
// grid == 0: one workgroup per point)
#define ROM_FUSED_DECL(T)                                                                              \
  int rom_fused_launch_##T(const FusedArgs& a, int prec, int split, int grid, int P, hipStream_t s);  \
  int rom_phased_cs_##T(const FusedArgs& a, int prec, int split, int P, hipStream_t s);               \
  int rom_phased_solve_##T(const FusedArgs& a, int P, hipStream_t s);                                  \
  int rom_fused_setup_##T();
ROM_FUSED_DECL(2)
ROM_FUSED_DECL(3)
ROM_FUSED_DECL(4)
ROM_FUSED_DECL(5)
ROM_FUSED_DECL(6)
ROM_FUSED_DECL(7)
ROM_FUSED_DECL(8)

// shared by the fused and phased dispatchers (rom_fused.hip)
int rom_fused_prepare(rom_model* h, int P, const double* Fbar, void* state, const rom_opts& o, int32_t* st_out,
                      int32_t* it_out, double* res_out, hipStream_t s, FusedArgs& a, int& split);
int rom_fused_launch(int T, const FusedArgs& a, int prec, int split, int grid, int P, hipStream_t s);
int rom_phased_cs(int T, const FusedArgs& a, int prec, int split, int P, hipStream_t s);
int rom_phased_solve(int T, const FusedArgs& a, int P, hipStream_t s);
bool rom_refines_abar(const rom_opts& o);
int rom_refine_abar(const rom_model* h, const FusedArgs& a, int split, int P, void* state, hipStream_t s);
int rom_refine_abar_phased(const rom_model* h, const FusedArgs& a, int split, int P, void* state, hipStream_t s);
