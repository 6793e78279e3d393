// Fused online solve, 5 column blocks of 16 (n + 5 <= 80).
#include "rom_fused_impl.h"

ROM_FUSED_DEFINE(5)
