// The one-pass opening and closing for uint16_t images (a translation unit of its own:
// its windows take long to compile).
#include "k_openclose_wave.h"

namespace morph {

hipError_t launch_openclose_wave_u16(const TileJob &job, hipStream_t stream)
{
    return launch_openclose_wave_t<uint16_t>(job, stream);
}

} // namespace morph
