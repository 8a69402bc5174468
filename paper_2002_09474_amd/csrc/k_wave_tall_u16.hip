// The wave kernel's tall form for uint16_t images (a translation unit of its own: the
// tall windows take long to compile).
#include "k_wave_tall.h"

namespace morph {

hipError_t launch_wave_tall_u16(const TileJob &job, hipStream_t stream)
{
    return launch_wave_tall_t<uint16_t>(job, stream);
}

hipError_t launch_batch_wave_tall_u16(const BatchTables &t, bool aligned, int grid,
                                     hipStream_t stream)
{
    return launch_batch_wave_tall_t<uint16_t>(t, aligned, grid, stream);
}

} // namespace morph
