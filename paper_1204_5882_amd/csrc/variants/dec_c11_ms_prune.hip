// Decoder variant: register-resident subtree 2^11, min-sum check update,
// pruning on, leaf-LLR dump off.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c11_ms_prune, 11, 0, true, false)
