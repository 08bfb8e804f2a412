// kb_wave2_k128.hip -- the two-word wavefront kernel (kb_wave2.h) with two
// beam slots per lane: beams of 65..128 slots on one wavefront per pair.
#include "kb_wave2.h"

namespace gedk {

const void *select_wave2_two_slots(int PL, bool small, bool complete, bool dir) {
    return w2::select_wave2_s<2>(PL, small, complete, dir);
}

}  // namespace gedk
