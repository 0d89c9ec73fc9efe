// Decoder variant: register-resident subtree 2^12, min-sum check update,
// pruning off, leaf-LLR dump on.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c12_ms_dump, 12, 0, false, true)
