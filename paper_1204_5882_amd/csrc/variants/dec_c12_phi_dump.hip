// Decoder variant: register-resident subtree 2^12, fixed-point phi-table check update,
// pruning off, leaf-LLR dump on.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c12_phi_dump, 12, 3, false, true)
