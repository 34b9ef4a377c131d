// KSG kernel instantiations with a top-k capacity of 16 (k <= 16).
// Parameters: KMAX, estimates per lane G, queries per lane QP, and the Z, Y
// and X column capacities.
#include "ksg_device.h"

namespace mte {

const dev::VariantEntry *variants_k16(int *n) {
    static const dev::VariantEntry v[] = {
    MTE_VARIANT_ENTRY(16, 8, 1, 8, 1, 1)
    MTE_VARIANT_ENTRY(16, 8, 2, 8, 1, 1)
    MTE_VARIANT_ENTRY(16, 4, 2, 8, 1, 1)
    MTE_VARIANT_ENTRY(16, 4, 2, 16, 1, 1)
    MTE_VARIANT_ENTRY(16, 4, 2, 32, 1, 1)
    MTE_VARIANT_ENTRY(16, 1, 2, 8, 1, 1)
    MTE_VARIANT_ENTRY(16, 1, 2, 16, 1, 1)
    MTE_VARIANT_ENTRY(16, 1, 2, 32, 1, 1)
    MTE_VARIANT_ENTRY(16, 2, 2, 32, 1, 16)
    MTE_VARIANT_ENTRY(16, 1, 2, 32, 8, 16)
    };
    *n = (int)(sizeof(v) / sizeof(v[0]));
    return v;
}

}  // namespace mte
