// Decoder variant: register-resident subtree 2^12, box-plus check update,
// pruning off, leaf-LLR dump off.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c12_bp, 12, 1, false, false)
