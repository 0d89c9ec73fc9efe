// Decoder variant: register-resident subtree 2^12, min-sum check update,
// pruning off, leaf-LLR dump off.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c12_ms, 12, 0, false, false)
