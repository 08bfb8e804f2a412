// kb_wave2_src128.hip -- the two-word wavefront kernel (kb_wave2.h) for
// undirected sources of 65..128 vertices (targets of up to 64): the mapping
// takes 32 words of bytes and row v_i of g1 is read once per level; one beam
// slot per lane up to K = 64, two up to 128.
#include "kb_wave2.h"

namespace gedk {

const void *select_wave2_wide_source(int slots, int PL, bool small, bool complete) {
    return slots == 1 ? w2::select_wave2_wide_src<1>(PL, small, complete)
                      : w2::select_wave2_wide_src<2>(PL, small, complete);
}

}  // namespace gedk
