// Fused online solve, 7 column blocks of 16 (n + 5 <= 112).
#include "rom_fused_impl.h"

ROM_FUSED_DEFINE(7)
