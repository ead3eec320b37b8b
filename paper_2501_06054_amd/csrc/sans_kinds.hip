// sans_kinds.hip -- instances of the per-model kernels for one group of
// models (SANS_KIND_GROUP = g: the kinds K with K % kKindGroups == g).  The
// build compiles this file once per group, in parallel.
#include "sans_kernels.hpp"

#ifndef SANS_KIND_GROUP
#error "SANS_KIND_GROUP must be defined (0 .. kKindGroups - 1)"
#endif

#define SANS_CAT2(a, b) a##b
#define SANS_CAT(a, b) SANS_CAT2(a, b)

namespace sans {

namespace {
template <int K>
void fill_group(KindFns* t)
{
    if constexpr (K < kNumKinds) {
        fill_kind<K>(t);
        fill_group<K + kKindGroups>(t);
    }
}
}  // namespace

void SANS_CAT(fill_kinds_, SANS_KIND_GROUP)(KindFns* t) { fill_group<SANS_KIND_GROUP>(t); }

}  // namespace sans
