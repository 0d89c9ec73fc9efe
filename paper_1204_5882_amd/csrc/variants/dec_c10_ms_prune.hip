// Decoder variant: register-resident subtree 2^10, min-sum check update,
// pruning on, leaf-LLR dump off.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c10_ms_prune, 10, 0, true, false)
