// Decoder variant: register-resident subtree 2^12, box-plus check update,
// pruning on, leaf-LLR dump on.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c12_bp_prune_dump, 12, 1, true, true)
