// FP64 and split-precision operator products of prisms (tags 4..7): one translation unit per element type and precision so
// that the product instantiations compile in parallel.
#include "fr_opmul.hpp"

namespace frd {

FR_OPMUL_INSTANCE(double, 4)
FR_OPMUL_INSTANCE(double, 5)
FR_OPMUL_INSTANCE(double, 6)
FR_OPMUL_INSTANCE(double, 7)
FR_SPLIT_INSTANCE(false, 4) FR_SPLIT_INSTANCE(true, 4)
FR_SPLIT_INSTANCE(false, 5) FR_SPLIT_INSTANCE(true, 5)
FR_SPLIT_INSTANCE(false, 6) FR_SPLIT_INSTANCE(true, 6)
FR_SPLIT_INSTANCE(false, 7) FR_SPLIT_INSTANCE(true, 7)

}  // namespace frd
