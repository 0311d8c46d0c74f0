// Library-internal entry points shared by the C ABI (api.cpp) and the request
// server (serve.cpp).  Not part of the public header.
#pragma once
#include <atomic>
#include <string>

#include "../../include/ofdft.h"

namespace ofdft_internal {

// Moves the atoms of a grid (same count and species) and rebuilds the phase
// tables, v_ext(G) and E_ion in place.  The resident density is kept.
ofdft_status set_positions(ofdft_grid *g, const double *pos);
// Runs the grid's later work on another context of the same device.  The
// caller guarantees that no work of the grid is in flight.
void bind_context(ofdft_grid *g, ofdft_ctx *ctx);
// Flag polled by the optimiser once per iteration (nullptr: none).
void set_cancel(ofdft_grid *g, const std::atomic<int> *flag);
// Sets the calling thread's ofdft_last_error() message.
void set_error(const std::string &msg);
int ctx_device(const ofdft_ctx *ctx);
// Whether the process already holds a tuned launch schedule for this grid's
// shape, precision, functional and single-density batches.
bool has_tuning(const ofdft_grid *g);
// Device bytes by which ofdft_energy_potential_multi led by g would grow g's
// allocations for a batch of n grids (workspace for n densities and the
// batch staging); 0 when they already suffice.
uint64_t multi_growth_bytes(const ofdft_grid *g, int n);

}  // namespace ofdft_internal
