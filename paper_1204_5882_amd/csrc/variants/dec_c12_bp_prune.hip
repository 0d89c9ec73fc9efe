// Decoder variant: register-resident subtree 2^12, box-plus check update,
// pruning on, leaf-LLR dump off.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c12_bp_prune, 12, 1, true, false)
