// Instantiation of the P64 kernels for every supported tile size.
#include "engine.h"

namespace lq {
const Ops *ops_p64(int nb) {
    switch (nb) {
    case 32: return Eng<32, P64>::ops();
    case 64: return Eng<64, P64>::ops();
    case 128: return Eng<128, P64>::ops();
    case 256: return Eng<256, P64>::ops();
    default: return nullptr;
    }
}
}  // namespace lq
