// Launchers of the fused online solve (one persistent kernel per step).
#pragma once
#include "rom_common.h"

int rom_fused_setup();
int rom_fused_tiles(int n);  // 16-column tiles of the padded system (n + 5 columns)
int rom_launch_step_fused(rom_model* h, int P, const double* Fbar, void* state, const rom_opts& o,
                          int32_t* st_out, int32_t* it_out, double* res_out, hipStream_t s);
int rom_launch_step_phased(rom_model* h, int P, const double* Fbar, void* state, const rom_opts& o,
                           int32_t* st_out, int32_t* it_out, double* res_out, hipStream_t s);
int rom_launch_shape_sensitivity(rom_model* h, int P, const double* Fbar, const void* state, double* out,
                                 hipStream_t s);

// rom_step_noalloc: the persistent fused form with its queue in static device
// memory (rom_noalloc_setup looks its address up once per device)
int rom_noalloc_setup(int device);
int rom_launch_step_noalloc(rom_model* h, int P, const double* Fbar, void* state, const rom_opts& o,
                            int32_t* st_out, int32_t* it_out, double* res_out, hipStream_t s);
