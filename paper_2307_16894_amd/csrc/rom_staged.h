// Launchers of the staged online solve (one kernel per stage).
#pragma once
#include "rom_common.h"

int rom_staged_setup();
int rom_launch_state_init(const rom_model* h, int P, const double* mu, void* state, hipStream_t s);
int rom_launch_step_staged(rom_model* h, int P, const double* Fbar, void* state, const rom_opts& o,
                           int32_t* st_out, int32_t* it_out, double* res_out, hipStream_t s);
int rom_launch_path_gather(int P, const double* paths, int max_steps, const int* nsteps, const int* step, double* Fbar,
                           int* active, hipStream_t s);
int rom_launch_path_advance(int P, const int* active, int* step, hipStream_t s);
int rom_launch_warm_samples(const rom_model* h, int P, const void* state, const float* X_feat, const double* r_before,
                            const int* status, float* X_out, float* Y_out, int* count, hipStream_t s);
int rom_launch_commit_trial(const rom_model* h, int P, const double* Fbar, void* state, const int* status,
                            hipStream_t s);
