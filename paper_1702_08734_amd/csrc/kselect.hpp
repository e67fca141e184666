// Selector sizing shared by the kernels.
#pragma once

#include <cstdint>

namespace mk {

constexpr int kMaxK = 1024;

// Wave-queue registers (64 entries each, a power of two) holding k entries.
inline int queue_regs(int k) {
    int r = 1;
    while (r * 64 < k) r *= 2;
    return r;
}

// Thread-queue length per wave-queue size.  Section 4.3 tunes t against k
// on Maxwell (2 for k <= 32, 3 for k <= 128, 4 for k <= 256, 8 for
// k <= 1024); here t is a power of two so that the thread-queue sort is a
// plain bitonic network on whole registers.
template <int KR>
struct SelParams;
template <> struct SelParams<1> { static constexpr int T = 2; };
template <> struct SelParams<2> { static constexpr int T = 2; };
template <> struct SelParams<4> { static constexpr int T = 4; };
template <> struct SelParams<8> { static constexpr int T = 4; };
template <> struct SelParams<16> { static constexpr int T = 8; };

}  // namespace mk
