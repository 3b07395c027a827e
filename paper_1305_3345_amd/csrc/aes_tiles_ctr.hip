// aes_tiles_ctr.hip -- encryption-side tile kernels (CTR and ECB encryption).
// Built with LLVM's default instruction scheduler.  Before CTR tiles computed
// the first two rounds' shared part once per group of counters, the max-ILP
// scheduler was 3% faster here; with that shared part it leaves round keys
// spilled to scratch, and the default scheduler gives the fastest CTR tiles
// on every key size (ECB encryption tiles lose 1-2% against max-ILP).
#include "tile_kernel.h"

namespace aesgpu {

bool tile_shape_supported(int nb, int wg) {
    return wg >= 64 && wg <= 1024 && wg % 64 == 0 && pick_tile_kernel<false>(nb, wg) != nullptr;
}

int launch_ctr_tiles(const Unit *d_units, uint32_t n_units, const aes_schedule_t *d_sched,
                     uint32_t n_sched, const uint32_t *d_timg, const uint8_t *d_in,
                     uint8_t *d_out, uint32_t *d_ctrs, const TileLaunch &cfg, int n_cu,
                     void *stream) {
    return launch_tiles<false>(d_units, n_units, d_sched, n_sched, d_timg, nullptr, d_in, d_out,
                               d_ctrs, cfg, n_cu, stream);
}

}  // namespace aesgpu
