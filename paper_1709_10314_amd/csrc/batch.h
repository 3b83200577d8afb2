// Descriptors of the batch kernels (batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smf {

constexpr int kMaxTiles = 4;                       // m-tiles per chain item (tile shape)
constexpr int kMaxChainThreads = 64 * 2 * kMaxTiles;

struct BatchField {
    const float* fac;     // FP32 factor records of the field's plan
    const float* tw;      // its FFT twiddles
    int64_t out_off;      // first element of the field in the packed output
    int n_theta, n_phi, order, m_top, m_rows, n_sets, s, even, log2h;
    int seed_off;         // Philox key = seed + seed_off
};

// Per-call entry of one field in the form with per-field seeds and output buffers.
struct BatchCall {
    uint64_t key;         // Philox key of the field
    float* out;           // the field's own [ring][phi] buffer
};

struct BatchArgs {
    const BatchField* fields;
    const BatchCall* call;         // per-field keys and buffers, or null: key seed + seed_off,
                                   // field at out + out_off (packed output)
    const uint32_t* chain_items;   // (field << 16) | group of `tiles` m-tiles
    const uint32_t* fft_items;     // (field << 16) | ring
    float* out;
    uint64_t seed;
    int tiles;                     // m-tiles per chain item: 1, 2 or 4
    int n_chain_items, n_fft_items;
};

hipError_t launch_batch(const BatchArgs& a, size_t lds, hipStream_t st);
// The same work in one cooperative launch with a grid barrier between the chain items and the
// ring items (grid_out: the workgroups launched); hipErrorCooperativeLaunchTooLarge when the
// device cannot hold a workgroup of the tile shape at once.
hipError_t launch_batch_persistent(const BatchArgs& a, size_t lds, hipStream_t st, int* grid_out);

}  // namespace smf
