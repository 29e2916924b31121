// Instantiation of the PB16 kernels for every supported tile size.
#include "engine.h"

namespace lq {
const Ops *ops_pb16(int nb) {
    switch (nb) {
    case 32: return Eng<32, PB16>::ops();
    case 64: return Eng<64, PB16>::ops();
    case 128: return Eng<128, PB16>::ops();
    case 256: return Eng<256, PB16>::ops();
    case 512: return Eng<512, PB16>::ops();
    default: return nullptr;
    }
}
}  // namespace lq
