/*
 * Bulk generator for the seeded synthetic inputs (synthon embedding tables).
 *
 * Same streams as workloads/gen.py: value n of a stream is
 * splitmix64(key + (n + 1) * 0x9E3779B97F4A7C15) (Steele, Lea and Flood,
 * OOPSLA 2014); a normal variate takes counters 2n and 2n+1 through the
 * Box-Muller transform (cosine branch). log and cos are evaluated with the same
 * series and the same operation order as the Python version, using only
 * correctly rounded IEEE double operations, so both produce identical bits.
 * Build with -ffp-contract=off (no fused multiply-add) to keep that true.
 *
 * Holds no arithmetic of the search method.
 */
#include <math.h>
#include <stdint.h>

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static inline double u01(uint64_t key, uint64_t ctr) {
  uint64_t x = mix64(key + (ctr + 1) * 0x9E3779B97F4A7C15ull);
  return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

static double det_log(double x) {
  int e;
  double m = frexp(x, &e);
  if (m < 0.7071067811865476) {
    m = m * 2.0;
    e = e - 1;
  }
  double s = (m - 1.0) / (m + 1.0);
  double s2 = s * s;
  double acc = 0.0;
  for (int n = 25; n >= 1; n -= 2) acc = acc * s2 + 1.0 / (double)n;
  return 2.0 * s * acc + (double)e * 0.6931471805599453;
}

static double det_cos_2pi(double v) {
  double w = v * 8.0;
  double octant = floor(w);
  double f = w - octant;
  int o = ((int)octant) & 7;
  double a = ((o & 1) ? (1.0 - f) : f) * (3.141592653589793 / 4.0);
  double a2 = a * a;
  double s = 0.0, c = 0.0, ts = a, tc = 1.0;
  for (int n = 0; n < 11; n++) {
    s = s + ts;
    c = c + tc;
    ts = -ts * a2 / (double)((2 * n + 2) * (2 * n + 3));
    tc = -tc * a2 / (double)((2 * n + 1) * (2 * n + 2));
  }
  switch (o) {
    case 0: return c;
    case 1: return s;
    case 2: return -s;
    case 3: return -c;
    case 4: return -c;
    case 5: return -s;
    case 6: return s;
    default: return c;
  }
}

/* out[i] = float32(N(0,1) value number offset+i of the stream with this key). */
void gen_normal_f32(uint64_t key, uint64_t offset, uint64_t n, float* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)n; i++) {
    uint64_t c = 2 * (offset + (uint64_t)i);
    double u1 = 1.0 - u01(key, c);
    double u2 = u01(key, c + 1);
    double r = sqrt(-2.0 * det_log(u1));
    out[i] = (float)(r * det_cos_2pi(u2));
  }
}
