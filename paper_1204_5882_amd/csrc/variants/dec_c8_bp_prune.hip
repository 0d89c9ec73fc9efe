// Decoder variant: register-resident subtree 2^8, box-plus check update,
// pruning on, leaf-LLR dump off.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c8_bp_prune, 8, 1, true, false)
