// Fused online solve, 4 column blocks of 16 (n + 5 <= 64).
#include "rom_fused_impl.h"

ROM_FUSED_DEFINE(4)
