// FP64 and split-precision operator products of hexahedra (tags 8..11): one translation unit per element type and precision so
// that the product instantiations compile in parallel.
#include "fr_opmul.hpp"

namespace frd {

FR_OPMUL_INSTANCE(double, 8)
FR_OPMUL_INSTANCE(double, 9)
FR_OPMUL_INSTANCE(double, 10)
FR_OPMUL_INSTANCE(double, 11)
FR_SPLIT_INSTANCE(false, 8) FR_SPLIT_INSTANCE(true, 8)
FR_SPLIT_INSTANCE(false, 9) FR_SPLIT_INSTANCE(true, 9)
FR_SPLIT_INSTANCE(false, 10) FR_SPLIT_INSTANCE(true, 10)
FR_SPLIT_INSTANCE(false, 11) FR_SPLIT_INSTANCE(true, 11)

}  // namespace frd
