// Kernel choice for one image or one batch group: each kernel family lives in a
// translation unit of its own (k_*.hip), which exports the launchers used here.
#include "morph_internal.h"

namespace morph {

hipError_t launch_tile_job(const TileJob &job, hipStream_t stream)
{
    switch (job.kind) {
    case KIND_ROWS: return launch_rows_kernel(job, stream);
    case KIND_STREAM: return job.coop ? launch_stream_coop(job, stream)
                                      : launch_stream_kernel(job, stream);
    case KIND_WAVE: return wave_tall(job) ? launch_wave_tall_kernel(job, stream)
                                          : launch_wave_kernel(job, stream);
    default: return launch_tile_kernel(job, stream);
    }
}

hipError_t launch_batch(const BatchTables &t, int kind, int variant, int waves, int dtype,
                        bool aligned, int grid, int lds, hipStream_t stream)
{
    switch (kind) {
    case KIND_ROWS: return launch_batch_rows(t, dtype, aligned, grid, stream);
    case KIND_WAVE: return variant ? launch_batch_wave_tall(t, dtype, aligned, grid, stream)
                                   : launch_batch_wave(t, dtype, aligned, grid, stream);
    case KIND_STREAM:
        if (variant == 2) return launch_batch_coop(t, dtype, waves, grid, lds, stream);
        return launch_batch_stream(t, variant != 0, dtype, aligned, grid, lds, stream);
    default: return launch_batch_tile(t, dtype, aligned, grid, lds, stream);
    }
}

hipError_t launch_wave_tall_kernel(const TileJob &job, hipStream_t stream)
{
    return job.dtype == 0 ? launch_wave_tall_u8(job, stream) : launch_wave_tall_u16(job, stream);
}

hipError_t launch_batch_wave_tall(const BatchTables &t, int dtype, bool aligned, int grid,
                                  hipStream_t stream)
{
    return dtype == 0 ? launch_batch_wave_tall_u8(t, aligned, grid, stream)
                      : launch_batch_wave_tall_u16(t, aligned, grid, stream);
}

hipError_t launch_openclose_wave(const TileJob &job, hipStream_t stream)
{
    return job.dtype == 0 ? launch_openclose_wave_u8(job, stream)
                          : launch_openclose_wave_u16(job, stream);
}

hipError_t launch_fused(const FusedTables &t, int dtype, bool aligned, int lds, hipStream_t stream)
{
    return dtype == 0 ? launch_fused_u8(t, aligned, lds, stream)
                      : launch_fused_u16(t, aligned, lds, stream);
}

} // namespace morph
