// Serving loop (continuous batching of independent systems).  Filled in
// by the serving milestone.
#include "hsma_internal.h"
