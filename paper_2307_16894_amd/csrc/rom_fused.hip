#include "rom_fused.h"

int rom_fused_setup() { return ROM_OK; }

int rom_launch_step_fused(rom_model*, int, const double*, void*, const rom_opts&, int32_t*, int32_t*,
                          double*, hipStream_t) {
  return ROM_EUNSUPPORTED;
}
