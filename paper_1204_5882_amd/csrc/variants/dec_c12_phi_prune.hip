// Decoder variant: register-resident subtree 2^12, fixed-point phi-table check update,
// pruning on, leaf-LLR dump off.
#include "sc_kernels.h"

POLAR_DECODE_VARIANT(polar_dec_c12_phi_prune, 12, 3, true, false)
