// ht_fill_rows.hip -- the fill kernel instantiated for one A-row count per tile, HT_FILL_ROWS,
// given on the compiler's command line (the build compiles this file once per row count, in
// parallel: each instantiates 16 kernel variants of store kind, vector width, candidate
// emission and record caching).
#include "ht_device.h"

#pragma clang fp contract(off)

#ifndef HT_FILL_ROWS
#error "HT_FILL_ROWS must be defined (1, 2, 4, 8, 16, 32 or 64)"
#endif

namespace ht {

template <>
hipError_t launch_fill_for_rows<HT_FILL_ROWS>(const DevGrid& g, const EvDesc& ev0, const EvDesc* evs,
                                              int n_ev, bool nt, bool vec, bool emit, bool long_lists,
                                              size_t lds, hipStream_t s)
{
  if (nt) return launch_fill_rows<HT_FILL_ROWS, true>(g, ev0, evs, n_ev, vec, emit, long_lists, lds, s);
  return launch_fill_rows<HT_FILL_ROWS, false>(g, ev0, evs, n_ev, vec, emit, long_lists, lds, s);
}

}  // namespace ht
