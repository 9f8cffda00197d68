// Library-internal helpers shared between the translation units of libheget.so (not exported
// through include/heget.h).
#pragma once

#include "heget.h"

// Product over the final-state parton species of (multiplicity)!: the identical-particle factor
// the paper puts on the phase space (remark after eq. phase-space).
double heget_detail_final_symmetry(heget_process_t p);
