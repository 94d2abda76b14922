// FP32 operator products of tetrahedra (tags 0..3): one translation unit per element type and precision so
// that the product instantiations compile in parallel.
#include "fr_opmul.hpp"

namespace frd {

FR_OPMUL_INSTANCE(float, 0)
FR_OPMUL_INSTANCE(float, 1)
FR_OPMUL_INSTANCE(float, 2)
FR_OPMUL_INSTANCE(float, 3)

}  // namespace frd
