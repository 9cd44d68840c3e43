// gce_search_split.hip -- search-kernel variants: split-precision path, disjoint phase bins.
#include "gce_search.h"

GCE_SEARCH_TABLE(gce::kPrecSplit, 0, search_table_split)
