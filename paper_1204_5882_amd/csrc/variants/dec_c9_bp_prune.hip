// Decoder variant: register-resident subtree 2^9, box-plus check update,
// pruning on, leaf-LLR dump off.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c9_bp_prune, 9, 1, true, false)
