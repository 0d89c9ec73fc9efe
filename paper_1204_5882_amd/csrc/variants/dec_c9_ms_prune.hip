// Decoder variant: register-resident subtree 2^9, min-sum check update,
// pruning on, leaf-LLR dump off.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c9_ms_prune, 9, 0, true, false)
