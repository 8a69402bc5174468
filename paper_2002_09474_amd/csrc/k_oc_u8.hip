// The one-pass opening and closing for uint8_t images (a translation unit of its own:
// its windows take long to compile).
#include "k_openclose_wave.h"

namespace morph {

hipError_t launch_openclose_wave_u8(const TileJob &job, hipStream_t stream)
{
    return launch_openclose_wave_t<uint8_t>(job, stream);
}

} // namespace morph
