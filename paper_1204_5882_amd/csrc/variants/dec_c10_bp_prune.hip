// Decoder variant: register-resident subtree 2^10, box-plus check update,
// pruning on, leaf-LLR dump off.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c10_bp_prune, 10, 1, true, false)
