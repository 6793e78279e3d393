// Fused online solve, 3 column blocks of 16 (n + 5 <= 48).
#include "rom_fused_impl.h"

ROM_FUSED_DEFINE(3)
