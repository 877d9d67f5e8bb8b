// Host-side check of the FP16 site-scale rule of the library's storage helpers: the
// reciprocal of a site's max |value| is finite for every finite, non-negative maximum,
// and zero (a zero site) below the smallest normal float. Prints one line per case and
// exits non-zero on a violation.
#include <cfloat>
#include <cmath>
#include <cstdio>

#include "core.hpp"

int main() {
    const float cases[] = {0.0f, 1e-45f, 1e-40f, 1.0e-39f, FLT_MIN * 0.5f, FLT_MIN, 2 * FLT_MIN, 1e-30f, 1.0f,
                           65504.0f, 1e30f, FLT_MAX};
    int bad = 0;
    for (float m : cases) {
        const float inv = sapdd::fp16_site_inv(m);
        const bool finite = std::isfinite(inv);
        const bool zero_below = m < FLT_MIN ? inv == 0.0f : inv > 0.0f;
        // a stored value is v * inv with |v| <= m: it must stay within [-1, 1] (up to rounding)
        const float top = m * inv;
        const bool bounded = top <= 1.0f + 1e-6f && !(top != top);
        std::printf("m=%.9g inv=%.9g m*inv=%.9g %s\n", m, inv, top, finite && zero_below && bounded ? "ok" : "BAD");
        bad += !(finite && zero_below && bounded);
    }
    return bad ? 1 : 0;
}
