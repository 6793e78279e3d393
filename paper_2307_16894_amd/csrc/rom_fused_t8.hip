// Fused online solve, 8 column blocks of 16 (n + 5 <= 128).
#include "rom_fused_impl.h"

ROM_FUSED_DEFINE(8)
