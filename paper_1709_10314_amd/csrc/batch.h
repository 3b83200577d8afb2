// Descriptors of the persistent batch kernel (batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smf {

struct BatchField {
    const float* fac;     // FP32 factor records of the field's plan
    const float* tw;      // its FFT twiddles
    int64_t out_off;      // first element of the field in the packed output
    int n_theta, n_phi, order, m_top, m_rows, s, even, log2h;
    int n_rec_items;      // chain items of this field
    int seed_off;         // Philox key = seed + seed_off
};

struct BatchArgs {
    const BatchField* fields;
    const uint32_t* items;   // (field << 16) | sub
    int* counters;           // [0] queue head, [1] error word, [2 + f] chain items done
    float* out;
    uint64_t seed;
    int n_fields, n_rec, n_items;
    int spin_limit;          // bound on the FFT items' waits (iterations of s_sleep)
};

hipError_t launch_batch(const BatchArgs& a, int grid, size_t lds, hipStream_t st);
hipError_t batch_max_blocks_per_cu(size_t lds, int* blocks);

}  // namespace smf
