// Kernel arguments of the fused online solve (shared by the per-tile-count
// translation units and the dispatcher).
#pragma once
#include "rom_common.h"

struct FusedArgs {
  int n, m, max_iter, fixed, commit;
  int max_sub;  // load-step cutting depth (0: plain step)
  double tol, inv_area;
  J2Params mp;
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
  double* fbc;       // committed Fbar [P][4]
};

// per tile-count entry points (rom_fused_t<T>.hip): launch with the given
// contraction precision, wave split (0 points, 1 tiles), and persistent grid
// (grid > 0: that many workgroups pulling from the work list in the args;
// grid == 0: one workgroup per point)
#define ROM_FUSED_DECL(T)                                                                              \
  int rom_fused_launch_##T(const FusedArgs& a, int prec, int split, int grid, int P, hipStream_t s);  \
  int rom_fused_setup_##T();
ROM_FUSED_DECL(2)
ROM_FUSED_DECL(3)
ROM_FUSED_DECL(4)
ROM_FUSED_DECL(5)
ROM_FUSED_DECL(6)
ROM_FUSED_DECL(7)
ROM_FUSED_DECL(8)
