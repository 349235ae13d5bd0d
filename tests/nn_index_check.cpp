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
// Raw-input staging (up to 48 channels: the network's float32 input and its gradients): the
// float f of the tile's halo rows -> (row, pixel, channel) and its LDS element; every (pixel,
// channel < cin_raw) written once, every padding channel zeroed once.
template <int TW> void raw_staging() {
    constexpr int R = 64 / TW, TH = 4 * R, HW = TW + 2, HH = TH + 2, NP = HW * HH;
    for (uint32_t cr = 1; cr <= 48; ++cr) {
        const uint32_t ci_pad = (cr + 15) / 16 * 16, ps = ci_pad + 8;
        static unsigned char hit[NP * 56];
        for (auto& h : hit) h = 0;
        const uint32_t seg = HW * cr, total = HH * seg;
        const float inv_cr = 1.0f / (float)cr, inv_seg = 1.0f / (float)seg;
        for (uint32_t f = 0; f < total; ++f) {
            const uint32_t row = div_by_inv(f, inv_seg), fr = f - mul24(row, seg);
            const uint32_t qx = div_by_inv(fr, inv_cr), c = fr - mul24(qx, cr);
            CHECK(row == f / seg && qx == (f % seg) / cr && c == (f % seg) % cr);
            const uint32_t idx = mul24(row * HW + qx, ps) + c;
            CHECK(idx == ((f / seg) * HW + (f % seg) / cr) * ps + (f % seg) % cr);
            CHECK(idx < (uint32_t)NP * ps && c < cr);
            hit[idx] += 1;
        }
        const uint32_t padc = ci_pad - cr;
        if (padc > 0) {
            const float inv_pad = 1.0f / (float)padc;
            for (uint32_t z = 0; z < NP * padc; ++z) {
                const uint32_t q = div_by_inv(z, inv_pad), c = cr + z - mul24(q, padc);
                CHECK(q == z / padc && c >= cr && c < ci_pad);
                hit[mul24(q, ps) + c] += 1;
            }
        }
        for (uint32_t q = 0; q < (uint32_t)NP; ++q)
            for (uint32_t c = 0; c < ps; ++c) CHECK(hit[q * ps + c] == (c < ci_pad ? 1 : 0));
    }
}

int main() {
    tw<32>();
    tw<16>();
    raw_staging<32>();
    raw_staging<16>();
    for (uint32_t d = 1; d <= 2048; ++d) {
        const float inv = 1.0f / (float)d;
        for (uint32_t x = 0; x < 16384; ++x) CHECK(div_by_inv(x, inv) == x / d);
    }
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
