// FP32 operator products of prisms (tags 4..7): one translation unit per element type and precision so
// that the product instantiations compile in parallel.
#include "fr_opmul.hpp"

namespace frd {

FR_OPMUL_INSTANCE(float, 4)
FR_OPMUL_INSTANCE(float, 5)
FR_OPMUL_INSTANCE(float, 6)
FR_OPMUL_INSTANCE(float, 7)

}  // namespace frd
