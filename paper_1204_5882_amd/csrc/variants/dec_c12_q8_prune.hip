// Decoder variant: register-resident subtree 2^12, saturating min-sum check update on 8-bit
// integers, pruning on, leaf-LLR dump off.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c12_q8_prune, 12, 4, true, false)
