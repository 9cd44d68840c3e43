// gce_search_fp64_overlap.hip -- search-kernel variants: FP64 path, 50%-overlapping phase bins.
#include "gce_search.h"

GCE_SEARCH_TABLE(gce::kPrecFp64, 1, search_table_fp64_overlap)
