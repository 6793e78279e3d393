// Fused online solve, 6 column blocks of 16 (n + 5 <= 96).
#include "rom_fused_impl.h"

ROM_FUSED_DEFINE(6)
