// Newton outcome histogram of one wavefront (device code of the reaction
// solve kernels).
#pragma once
#include "misdc_impl.h"

namespace misdc {

// Adds the outcomes of the wavefront's valid lanes to one set of the
// histogram (code > 0: converged after code linear solves; code < 0: not
// converged).  Every lane of the wavefront must call it; the first lane
// issues one atomic per distinct bin, so a wavefront whose cells took two
// or three different iteration counts costs two or three atomics.
__device__ inline void wave_hist_add(unsigned long long* set, bool valid, int code) {
    const int bin = code <= 0 ? 0 : (code < NEWTON_HIST_BINS - 1 ? code : NEWTON_HIST_BINS - 1);
    unsigned long long rem = __ballot(valid);
    while (rem) {
        const int lead = __ffsll((long long)rem) - 1;
        const int b = __shfl(bin, lead);
        const unsigned long long same = __ballot(valid && bin == b);
        if ((threadIdx.x & 63) == 0) atomicAdd(&set[b], (unsigned long long)__popcll(same));
        rem &= ~same;
    }
}

}  // namespace misdc
