// One instantiation of the kernels: precision LQ_P and tile size LQ_NB are
// given on the compiler command line, so every (precision, tile size) pair is
// its own translation unit and they compile in parallel.
#include "engine.h"

#if !defined(LQ_P) || !defined(LQ_NB)
#error "compile with -DLQ_P=<0|1|2> -DLQ_NB=<tile size>"
#endif

namespace lq {
template <> const Ops *eng_ops<LQ_NB, LQ_P>() { return Eng<LQ_NB, LQ_P>::ops(); }
}  // namespace lq
