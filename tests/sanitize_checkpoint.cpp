// Host test of the learned-closure checkpoint format and normalisation check
// (paper_2605_19796_amd/csrc/kcf_checkpoint.h), built with the address and undefined-behaviour
// sanitizers by tests/test_host_sanitize.py: a round trip, every short length, lengths past the
// end, single flipped bytes, random garbage, and statistics with zero, negative, infinite and
// NaN entries. Exits 0 when every case gives the expected verdict.
#include <cmath>
#include <cstdio>
#include <limits>
#include <random>
#include <vector>

#include "kcf_checkpoint.h"

using namespace kcf::ckpt;

static int failures = 0;

static void expect(bool ok, const char* what, size_t a = 0) {
  if (!ok) {
    std::printf("FAIL: %s (%zu)\n", what, a);
    ++failures;
  }
}

// Decodes a copy of exactly n bytes, so that any read past the end is caught.
static const char* decode_copy(const std::vector<unsigned char>& src, size_t n, int64_t* step,
                               std::vector<float>& pmv, std::vector<float>& norm) {
  std::vector<unsigned char> b(src.begin(), src.begin() + (long)std::min(n, src.size()));
  b.resize(n, 0x5a);
  return decode(n ? b.data() : nullptr, n, step, pmv.data(), norm.data());
}

int main() {
  std::mt19937_64 rng(20251203);
  std::uniform_real_distribution<float> U(-2.f, 2.f);
  std::vector<float> pmv(3 * kCkParams), norm(kCkNorm);
  for (float& v : pmv) v = U(rng);
  for (float& v : norm) v = U(rng);
  for (int i = 0; i < 14; ++i) norm[14 + i] = 0.5f + std::fabs(norm[14 + i]);
  for (int i = 0; i < 6; ++i) norm[34 + i] = 0.5f + std::fabs(norm[34 + i]);
  expect(check_norm(norm.data()) == nullptr, "valid statistics rejected");

  const std::vector<unsigned char> good = encode(123456789, pmv.data(), norm.data());
  expect(good.size() == kSize, "encoded size", good.size());
  int64_t step = -1;
  std::vector<float> p2(3 * kCkParams), n2(kCkNorm);
  expect(decode_copy(good, good.size(), &step, p2, n2) == nullptr, "round trip rejected");
  expect(step == 123456789 && p2 == pmv && n2 == norm, "round trip changed the state");

  // every length shorter than a checkpoint, and a few longer ones
  for (size_t n = 0; n < kSize; n += (n < 64 ? 1 : 997))
    expect(decode_copy(good, n, &step, p2, n2) != nullptr, "short checkpoint accepted", n);
  expect(decode_copy(good, kSize - 1, &step, p2, n2) != nullptr, "kSize - 1 accepted");
  for (size_t extra : {1, 8, 4096})
    expect(decode_copy(good, kSize + extra, &step, p2, n2) != nullptr, "long file accepted",
           extra);

  // one flipped byte anywhere: the magic or the hash no longer matches
  std::uniform_int_distribution<size_t> pos(0, kSize - 1);
  for (int t = 0; t < 2000; ++t) {
    std::vector<unsigned char> b = good;
    const size_t i = t < 16 ? (size_t)t : (t < 24 ? kSize - 1 - (size_t)(t - 16) : pos(rng));
    b[i] ^= (unsigned char)(1u << (t % 8));
    expect(decode_copy(b, b.size(), &step, p2, n2) != nullptr, "flipped byte accepted", i);
  }
  // random garbage of random sizes, including the checkpoint size
  std::uniform_int_distribution<int> byte(0, 255);
  for (int t = 0; t < 200; ++t) {
    const size_t n = t % 4 == 0 ? kSize : (size_t)(rng() % (2 * kSize));
    std::vector<unsigned char> b(n);
    for (auto& c : b) c = (unsigned char)byte(rng);
    expect(decode_copy(b, n, &step, p2, n2) != nullptr, "garbage accepted", n);
  }
  // a rejected checkpoint leaves the outputs alone
  {
    std::vector<float> p3(3 * kCkParams, 7.f), n3(kCkNorm, 7.f);
    int64_t s3 = 7;
    std::vector<unsigned char> b = good;
    b[100] ^= 1;
    decode_copy(b, b.size(), &s3, p3, n3);
    expect(s3 == 7 && p3[0] == 7.f && n3[0] == 7.f, "outputs written on failure");
  }

  // statistics with a bad scale or mean in every slot that is checked
  const float bad[] = {0.f, -1.f, std::numeric_limits<float>::infinity(),
                       std::numeric_limits<float>::quiet_NaN()};
  for (int slot : {0, 13, 14, 27, 28, 33, 34, 39}) {
    const bool is_scale = (slot >= 14 && slot < 28) || slot >= 34;
    for (float v : bad) {
      if (!is_scale && (v == 0.f || v == -1.f)) continue;  // any finite mean is allowed
      std::vector<float> nn = norm;
      nn[slot] = v;
      expect(check_norm(nn.data()) != nullptr, "bad statistic accepted", (size_t)slot);
    }
  }
  // open envelope sides are allowed
  {
    std::vector<float> nn = norm;
    nn[40] = -std::numeric_limits<float>::infinity();
    nn[67] = std::numeric_limits<float>::infinity();
    expect(check_norm(nn.data()) == nullptr, "open envelope rejected");
  }
  std::printf("%s: %d failure(s)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
