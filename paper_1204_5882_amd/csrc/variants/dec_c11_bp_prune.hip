// Decoder variant: register-resident subtree 2^11, box-plus check update,
// pruning on, leaf-LLR dump off.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c11_bp_prune, 11, 1, true, false)
