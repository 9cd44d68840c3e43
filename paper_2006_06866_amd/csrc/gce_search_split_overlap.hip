// gce_search_split_overlap.hip -- search-kernel variants: split-precision path, 50%-overlapping phase bins.
#include "gce_search.h"

GCE_SEARCH_TABLE(gce::kPrecSplit, 1, search_table_split_overlap)
