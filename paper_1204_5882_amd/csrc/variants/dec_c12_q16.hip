// Decoder variant: register-resident subtree 2^12, fixed-point saturating min-sum check update,
// pruning off, leaf-LLR dump off.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c12_q16, 12, 2, false, false)
