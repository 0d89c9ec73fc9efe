// Decoder variant: register-resident subtree 2^12, fixed-point saturating min-sum check update,
// pruning off, leaf-LLR dump on.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c12_q16_dump, 12, 2, false, true)
