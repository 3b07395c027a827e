// aes_tiles_dec.hip -- decryption-side tile kernels (CBC and ECB decryption).
// Built with LLVM's max-ILP instruction scheduler, two blocks per lane.
// Measured on 4 KiB pages with each variant's launches interleaved in one
// process, on two boxes: 2.2% and 4.0% faster than the iterative ILP
// scheduler on AES-128, 0.8% and 3.4% on AES-256 (the default scheduler:
// 1.4% / 1.6% on one box); one kernel serves every key size of a batch,
// since plans never see the schedules.
#include "tile_kernel.h"

namespace aesgpu {

int launch_cbcdec_tiles(const Unit *d_units, uint32_t n_units, const aes_schedule_t *d_sched,
                        uint32_t n_sched, const uint32_t *d_timg, const void *d_preds,
                        const uint8_t *d_in, uint8_t *d_out, uint32_t *d_ctrs,
                        const TileLaunch &cfg, int n_cu, void *stream) {
    return launch_tiles<true>(d_units, n_units, d_sched, n_sched, d_timg, d_preds, d_in, d_out,
                              d_ctrs, cfg, n_cu, stream);
}

}  // namespace aesgpu
