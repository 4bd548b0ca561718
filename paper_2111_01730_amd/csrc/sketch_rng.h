// Counter-based random values of the construction's sketches, the same bits on the host
// and the device: an integer hash (splitmix64 finalizer) of (seed, row, column) picks
// one of the four values (+-1 +- j) / sqrt(2).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hodbf {

__host__ __device__ inline uint64_t sketch_hash(uint64_t seed, uint64_t r, uint64_t g) {
  uint64_t z = seed ^ (r * 0x9E3779B97F4A7C15ull) ^ (g * 0xD1B54A32D192ED03ull);
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

// real and imaginary parts: bit 0 and bit 1 of the hash choose the signs
__host__ __device__ inline void sketch_parts(uint64_t seed, uint64_t r, uint64_t g, double &re,
                                             double &im) {
  const uint64_t h = sketch_hash(seed, r, g);
  const double s = 0.70710678118654752440;
  re = (h & 1) ? -s : s;
  im = (h & 2) ? -s : s;
}

}  // namespace hodbf
