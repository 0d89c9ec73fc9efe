// Decoder variant: register-resident subtree 2^8, min-sum check update,
// pruning on, leaf-LLR dump off.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c8_ms_prune, 8, 0, true, false)
