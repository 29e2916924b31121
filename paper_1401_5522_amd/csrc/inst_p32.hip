// Instantiation of the P32 kernels for every supported tile size.
#include "engine.h"

namespace lq {
const Ops *ops_p32(int nb) {
    switch (nb) {
    case 32: return Eng<32, P32>::ops();
    case 64: return Eng<64, P32>::ops();
    case 128: return Eng<128, P32>::ops();
    case 256: return Eng<256, P32>::ops();
    case 512: return Eng<512, P32>::ops();
    default: return nullptr;
    }
}
}  // namespace lq
