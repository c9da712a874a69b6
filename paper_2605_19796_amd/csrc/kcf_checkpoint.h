// Host-only pieces of the learned-closure state: the checkpoint format and the validation of
// standardisation statistics. No HIP: this header is also compiled on its own with the address
// and undefined-behaviour sanitizers by the tests (tests/sanitize_checkpoint.cpp).
//
// Checkpoint layout (little endian, 8 + 8 + 3 * 4 * kCkParams + 4 * kCkNorm + 8 bytes):
//   "KCFMLP01" | int64 Adam step | float params[P] | float m[P] | float v[P] |
//   float norm[68] | uint64 FNV-1a hash of every byte before it
#pragma once

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace kcf {
namespace ckpt {

constexpr int kCkParams = 9670;  // network parameters
constexpr int kCkNorm = 68;      // standardisation statistics and envelope
constexpr char kMagic[9] = "KCFMLP01";
constexpr size_t kSize = 8 + 8 + 3 * (size_t)kCkParams * 4 + (size_t)kCkNorm * 4 + 8;

inline uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

// The checkpoint bytes of a state: pmv holds params, m and v (3 * kCkParams floats).
inline std::vector<unsigned char> encode(int64_t step, const float* pmv, const float* norm) {
  std::vector<unsigned char> out;
  out.reserve(kSize);
  auto put = [&](const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    out.insert(out.end(), b, b + n);
  };
  put(kMagic, 8);
  put(&step, sizeof(step));
  put(pmv, 3 * (size_t)kCkParams * 4);
  put(norm, (size_t)kCkNorm * 4);
  const uint64_t h = fnv1a(out.data(), out.size());
  put(&h, sizeof(h));
  return out;
}

// Parses n bytes; on success fills step, pmv (3 * kCkParams floats) and norm (kCkNorm floats)
// and returns nullptr, otherwise returns the reason and leaves the outputs untouched.
inline const char* decode(const unsigned char* in, size_t n, int64_t* step, float* pmv,
                          float* norm) {
  if (n != kSize) return "checkpoint has the wrong size";
  if (std::memcmp(in, kMagic, 8) != 0) return "not a checkpoint";
  uint64_t h;
  std::memcpy(&h, in + kSize - 8, 8);
  if (h != fnv1a(in, kSize - 8)) return "checkpoint checksum mismatch";
  std::memcpy(step, in + 8, 8);
  std::memcpy(pmv, in + 16, 3 * (size_t)kCkParams * 4);
  std::memcpy(norm, in + 16 + 3 * (size_t)kCkParams * 4, (size_t)kCkNorm * 4);
  return nullptr;
}

// Standardisation statistics [x_mu 14 | x_sd 14 | y_mu 6 | y_sd 6 | x_lo 14 | x_hi 14]:
// nullptr when every scale is positive and finite and every mean finite, else the reason.
// The envelope bounds may be infinite (an open side).
inline const char* check_norm(const float* norm) {
  for (int i = 0; i < 14; ++i)
    if (!(norm[14 + i] > 0) || !std::isfinite(norm[14 + i]) || !std::isfinite(norm[i]))
      return "input scales must be finite and > 0, and means finite";
  for (int i = 0; i < 6; ++i)
    if (!(norm[34 + i] > 0) || !std::isfinite(norm[34 + i]) || !std::isfinite(norm[28 + i]))
      return "target scales must be finite and > 0, and means finite";
  return nullptr;
}

}  // namespace ckpt
}  // namespace kcf
