// Host check of the tiled convolution's index helpers (csrc/nn_index.hpp) against the plain
// formulas they replace, over every tile shape, channel padding and stride the kernel accepts.
#include <cstdio>
#include <cstdint>
#include "nn_index.hpp"
using namespace casclb::nn;
static long bad = 0, n = 0;
#define CHECK(c) do { ++n; if (!(c)) { if (bad++ < 10) printf("FAIL %s line %d\n", #c, __LINE__); } } while (0)
template <int TW> void tw() {
    constexpr int R = 64 / TW, TH = 4 * R, HW = TW + 2, HH = TH + 2, NP = HW * HH, TPR = TW / 16;
    using D = SmallDiv<HW, NP>;
    for (uint32_t q = 0; q < (uint32_t)NP; ++q) CHECK(D::div(q) == q / HW);
    for (uint32_t ci_pad = 16; ci_pad <= 128; ci_pad += 8) {
        const uint32_t cpp = ci_pad / 8;
        const float inv = 1.0f / (float)cpp;
        for (uint32_t e = 0; e < NP * cpp; ++e) {
            uint32_t q, c0;
            chunk_of(e, cpp, inv, q, c0);
            CHECK(q == e / cpp && c0 == (e % cpp) * 8);
        }
        const uint32_t ps = ci_pad + 8;
        const uint32_t ktot = 9 * ci_pad, kpad = (ktot + 31) / 32 * 32;
        for (int wave = 0; wave < 4; ++wave)
            for (int grp = 0; grp < 4; ++grp)
                for (int col = 0; col < 16; ++col) {
                    TapCursor kc;
                    kc.start(8 * grp, ci_pad);
                    for (uint32_t kq = 0; kq < kpad; kq += 32) {
                        const uint32_t k0 = kq + 8 * grp;
                        if (k0 < ktot) {
                            CHECK(kc.tap == k0 / ci_pad && kc.c == k0 % ci_pad);
                            const uint32_t tap = k0 / ci_pad, c0 = k0 - tap * ci_pad;
                            const uint32_t dy = tap / 3, dx = tap - 3 * dy;
                            const uint32_t ndy = tap_row(kc.tap), ndx = kc.tap - 3 * ndy;
                            CHECK(ndy == dy && ndx == dx);
                            for (int t = 0; t < 4; ++t) {
                                const uint32_t lp_old = (wave * R + t / TPR) * HW + 16 * (t % TPR) + col;
                                const uint32_t old = (lp_old + dy * HW + dx) * ps + c0;
                                const uint32_t neu = mul24(lp_old, ps) + mul24(ndy * HW + ndx, ps) + kc.c;
                                CHECK(old == neu);
                                CHECK(neu + 8 <= (uint32_t)NP * ps);   // inside the staged tile
                            }
                        }
                        kc.advance32(ci_pad);
                    }
                }
    }
}
int main() {
    tw<32>();
    tw<16>();
    for (uint32_t h = 8; h <= 512; h *= 2)
        for (uint32_t w = 16; w <= 512; w *= 2)
            for (uint32_t cs : {16u, 24u, 48u, 96u, 128u, 136u, 9u, 5u})
                for (uint32_t img = 0; img < 16; img += 5) {
                    if ((int64_t)16 * h * w * (cs + 8) >= (int64_t)1 << 31) continue;
                    const uint32_t co = cs >= 32 ? 16 : 0;
                    const PixelOffsets p = pixel_offsets(img, h, w, cs, co);
                    for (uint32_t y = 0; y < h; y += (h > 64 ? 7 : 1))
                        for (uint32_t x = 0; x < w; x += (w > 64 ? 5 : 1))
                            for (uint32_t c = 0; c < 8; c += 7) {
                                const int64_t old = (((int64_t)img * h + y) * w + x) * cs + co + c;
                                CHECK((int64_t)p.at(y, x, c) == old);
                            }
                }
    printf("%ld checks, %ld failures\n", n, bad);
    return bad != 0;
}
