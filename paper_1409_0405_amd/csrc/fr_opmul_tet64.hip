// FP64 and split-precision operator products of tetrahedra (tags 0..3): one translation unit per element type and precision so
// that the product instantiations compile in parallel.
#include "fr_opmul.hpp"

namespace frd {

FR_OPMUL_INSTANCE(double, 0)
FR_OPMUL_INSTANCE(double, 1)
FR_OPMUL_INSTANCE(double, 2)
FR_OPMUL_INSTANCE(double, 3)
FR_SPLIT_INSTANCE(false, 0) FR_SPLIT_INSTANCE(true, 0)
FR_SPLIT_INSTANCE(false, 1) FR_SPLIT_INSTANCE(true, 1)
FR_SPLIT_INSTANCE(false, 2) FR_SPLIT_INSTANCE(true, 2)
FR_SPLIT_INSTANCE(false, 3) FR_SPLIT_INSTANCE(true, 3)

}  // namespace frd
