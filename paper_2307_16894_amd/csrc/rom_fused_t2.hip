// Fused online solve, 2 column blocks of 16 (n + 5 <= 32).
#include "rom_fused_impl.h"

ROM_FUSED_DEFINE(2)
