/* Host (CPU) twin of synth/philox.py and synth/csrc/synth_gen.hip: the seeded
 * synthetic value of element e of tensor (seed, tensor id), computed in C so
 * that large test inputs (whole blocks of a 4-billion-element operand, or
 * thousands of sampled rows) can be generated in seconds.  No part of the
 * contraction method lives here.
 *
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the two value maps:
 *   uniform [-1,1): 53 high bits of (w1:w0) of the block at counter
 *                   (e_lo, e_hi, 0, 0), scaled by 2^-52, minus 1;
 *   normal:         (sum of the twelve words of the blocks at counters
 *                   (e_lo, e_hi, d, 0), d = 0,1,2) * 2^-32 - 6.
 * Both are exact in binary64; a scale other than 1 is applied as one binary64
 * multiply.  Built with -ffp-contract=off.
 */
#include <stdint.h>

typedef struct {
  uint32_t x, y, z, w;
} u4;

static u4 philox4x32_10(u4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * c.x;
    const uint64_t p1 = (uint64_t)M1 * c.z;
    const u4 n = {(uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
                  (uint32_t)p0};
    c = n;
  }
  return c;
}

static double value_at(uint64_t e, uint32_t seed, uint32_t tid, int dist, double scale) {
  const uint32_t elo = (uint32_t)e, ehi = (uint32_t)(e >> 32);
  double x;
  if (dist == 0) {
    const u4 c = {elo, ehi, 0u, 0u};
    const u4 w = philox4x32_10(c, seed, tid);
    const uint64_t k = (((uint64_t)w.y << 32) | w.x) >> 11;
    x = (double)k * 0x1p-52 - 1.0;
  } else {
    uint64_t s = 0;
    for (uint32_t d = 0; d < 3; ++d) {
      const u4 c = {elo, ehi, d, 0u};
      const u4 w = philox4x32_10(c, seed, tid);
      s += (uint64_t)w.x + w.y + w.z + w.w;
    }
    x = (double)s * 0x1p-32 - 6.0;
  }
  return scale != 1.0 ? x * scale : x;
}

/* out[i] = value of element idx[i], i < n.  Returns 0, or -1 for an unknown dist. */
int synth_host_values(const int64_t* idx, int64_t n, uint32_t seed, uint32_t tensor_id, int dist,
                      double scale, double* out) {
  if (dist != 0 && dist != 1) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = value_at((uint64_t)idx[i], seed, tensor_id, dist, scale);
  return 0;
}

/* out[i] = value of element first + i, i < n. */
int synth_host_fill(double* out, int64_t n, int64_t first, uint32_t seed, uint32_t tensor_id, int dist,
                    double scale) {
  if (dist != 0 && dist != 1) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = value_at((uint64_t)(first + i), seed, tensor_id, dist, scale);
  return 0;
}
