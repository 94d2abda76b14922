// FP32 operator products of hexahedra (tags 8..11): one translation unit per element type and precision so
// that the product instantiations compile in parallel.
#include "fr_opmul.hpp"

namespace frd {

FR_OPMUL_INSTANCE(float, 8)
FR_OPMUL_INSTANCE(float, 9)
FR_OPMUL_INSTANCE(float, 10)
FR_OPMUL_INSTANCE(float, 11)

}  // namespace frd
