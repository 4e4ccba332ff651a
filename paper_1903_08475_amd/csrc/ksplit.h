// K ranges of the split moment contraction (Sec. 4.3 step 2 split over the
// angular cells).  Plain C++, no HIP: the CPU tests compile it on its own.
#pragma once

namespace mpg {

// K cells per split when kang cells are split `splitk` ways in multiples of
// `step`: the smallest multiple of step whose splitk-fold covers kang, so
// split z covers [z*chunk, min(kang, (z+1)*chunk)) and the splits together
// cover every cell (trailing splits may be empty).
inline int ksplit_chunk(int kang, int splitk, int step) {
    const int per = (kang + splitk - 1) / splitk;
    return (per + step - 1) / step * step;
}

}  // namespace mpg
