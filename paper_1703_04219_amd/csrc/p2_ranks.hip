// The launcher tables of one subset of the ranks.  The build compiles this
// file once per subset, with P2_SHARD_RANKS(X) defined as X(r) for each rank
// r of the subset, so that the subsets compile in parallel.  Each rank of
// P2_RANKS belongs to exactly one subset: a rank in none leaves its table
// undefined and one in two defines it twice, and either fails the link.
#include "p2_rank_impl.h"

#ifndef P2_SHARD_RANKS
#error "P2_SHARD_RANKS(X) must name the ranks this object is built for"
#endif

namespace p2 {

P2_SHARD_RANKS(P2_DEFINE_RANK)

}  // namespace p2
