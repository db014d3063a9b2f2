// Host check of the library's signed root (device_common.h): the rounding
// step must turn any start value within one ulp of the correctly rounded
// root into that root, for every integer squared distance up to 2^22 and
// for the +-INT32_MAX markers.  The start value is the correctly rounded
// root moved by `g_shift` ulps (-1, 0, +1), standing in for the hardware
// root's error.  Prints the number of mismatches; exit status 1 if any.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

static int g_shift = 0;
static float start_value(float a) {
  const float c = std::sqrt(a);  // IEEE: correctly rounded
  if (c == 0.0f || std::isinf(c)) return c;  // the hardware is exact here
  int32_t b;
  std::memcpy(&b, &c, 4);
  b += g_shift;
  float r;
  std::memcpy(&r, &b, 4);
  return r;
}
#define PCSDF_HOST_ROOT_START(a) start_value(a)
#include "hip/hip_runtime.h"
#include "../../paper_2201_05058_amd/csrc/device_common.h"

int main() {
  long bad = 0;
  const float hf = 0.02f;
  for (g_shift = -1; g_shift <= 1; ++g_shift) {
    for (int32_t x = 0; x <= (1 << 22); ++x) {
      const float want = std::sqrt((float)x);
      if (pcsdf::sqrt_rn_nonneg((float)x) != want) ++bad;
      // the signed metres of x and -x
      const float m = hf * want;
      const float fp = pcsdf::ssq_to_metres(x, hf);
      const float fn = pcsdf::ssq_to_metres(-x, hf);
      if (fp != m || std::signbit(fp)) ++bad;
      if (x > 0 && fn != -m) ++bad;
    }
    if (pcsdf::ssq_to_metres(INT32_MAX, hf) != INFINITY) ++bad;
    if (pcsdf::ssq_to_metres(-INT32_MAX, hf) != -INFINITY) ++bad;
  }
  std::printf("mismatches %ld\n", bad);
  return bad ? 1 : 0;
}
