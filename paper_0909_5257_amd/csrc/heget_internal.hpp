// Library-internal helpers shared between the translation units of libheget.so (not exported
// through include/heget.h).
#pragma once

#include "heget.h"

// Product over the final-state parton species of (multiplicity)!: the identical-particle factor
// the paper puts on the phase space (remark after eq. phase-space).
double heget_detail_final_symmetry(heget_process_t p);

// heget_matrix_elements_helicity; with allow_sort == false the events are never sorted by chirality
// pattern (no work space is taken: the sampled kernel runs over the events in their own order).
heget_status heget_detail_matrix_elements_helicity(heget_process_t p, const double* momenta, const int32_t* helicity,
                                                   int64_t n_events, double alpha_s, double* me2, void* stream,
                                                   bool allow_sort);
