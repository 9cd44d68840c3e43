// gce_search_fp64.hip -- search-kernel variants: FP64 path, disjoint phase bins.
#include "gce_search.h"

GCE_SEARCH_TABLE(gce::kPrecFp64, 0, search_table_fp64)
