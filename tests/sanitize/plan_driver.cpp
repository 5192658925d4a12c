// Host sanitizer run of the library's planning (test infrastructure):
// sd7_plan on valid frame sets (one frame, 64 mixed frames, empty scenes,
// frames for both binners, the largest image side) and on every kind of
// invalid argument it must refuse.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side by tests/test_sanitize_host.py;
// no GPU is touched.  Exit status: the number of failed checks.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "sd7.h"

static float dummy[16];

static sd7_frame frame(int64_t n, int W, int H)
{
    sd7_frame f;
    std::memset(&f, 0, sizeof f);
    f.scene.mu_p = f.scene.mu_t = f.scene.mu_d = f.scene.L = f.scene.alpha = f.scene.sh = dummy;
    f.scene.n = n;
    f.view.R_wc[0] = f.view.R_wc[4] = f.view.R_wc[8] = 1.0f;
    f.view.W = W;
    f.view.H = H;
    f.view.fx = f.view.fy = 100.0f;
    f.view.cx = 0.5f * W;
    f.view.cy = 0.5f * H;
    f.image = f.final_T = dummy;
    f.last = reinterpret_cast<uint32_t*>(dummy);
    return f;
}

static int failures = 0;

static void expect_ok(const char* what, const std::vector<sd7_frame>& fr, int64_t cap)
{
    sd7_layout L;
    const sd7_status s = sd7_plan(fr.data(), (int)fr.size(), cap, &L);
    bool ok = s == SD7_OK && L.nframes == (int)fr.size() && L.pair_capacity == cap;
    int64_t g = 0;
    for (size_t f = 0; ok && f < fr.size(); ++f) {
        ok = L.g0[f] == g;
        g += fr[f].scene.n;
    }
    const size_t offs[] = {L.off_table, L.off_counts, L.off_mu_c, L.off_cov_c, L.off_alpha_c, L.off_splat,
                           L.off_rect, L.off_depth_key, L.off_order, L.off_pair_g, L.off_ranges, L.off_d_splat,
                           L.off_d_mu_c, L.off_d_cov_c, L.off_d_alpha_c, L.off_scratch};
    for (size_t o : offs) ok = ok && o % 256 == 0 && o <= L.bytes;
    ok = ok && L.n_total == g;
    std::printf("%-44s %s (%zu bytes)\n", what, ok ? "ok" : "FAILED", ok ? L.bytes : (size_t)0);
    failures += !ok;
}

static void expect_einval(const char* what, const std::vector<sd7_frame>& fr, int nf, int64_t cap)
{
    sd7_layout L;
    const sd7_status s = sd7_plan(nf ? fr.data() : nullptr, nf, cap, &L);
    const char* msg = sd7_last_error();
    const bool ok = s == SD7_EINVAL && msg && std::strlen(msg) > 0;
    std::printf("%-44s %s: %s\n", what, ok ? "refused" : "NOT REFUSED", msg ? msg : "(no message)");
    failures += !ok;
}

int main()
{
    expect_ok("one frame", {frame(1000, 64, 48)}, 1 << 16);
    std::vector<sd7_frame> mix;
    for (int f = 0; f < SD7_MAX_FRAMES; ++f) mix.push_back(frame(1000 + 977 * f, 16 + 37 * f, 9 + 23 * f));
    expect_ok("64 mixed frames", mix, 1 << 20);
    expect_ok("empty scenes", {frame(0, 64, 48), frame(5, 1, 1), frame(0, 3, 3)}, 0);
    expect_ok("frame above the counting binner's size", {frame(4096, 2912, 2912), frame(100, 64, 64)}, 1 << 18);
    expect_ok("largest side", {frame(10, SD7_MAX_DIM, 1), frame(10, 1, SD7_MAX_DIM)}, 4096);
    expect_ok("largest pair arena", {frame(10, 32, 32)}, ((int64_t)1 << 31) - 1 - SD7_PAIR_ROUND);

    std::vector<sd7_frame> one = {frame(100, 64, 48)};
    expect_einval("no frames", one, 0, 1024);
    std::vector<sd7_frame> many(SD7_MAX_FRAMES + 1, frame(10, 8, 8));
    expect_einval("too many frames", many, SD7_MAX_FRAMES + 1, 1024);
    auto bad = [&](const char* what, void (*edit)(sd7_frame&), int64_t cap = 1024) {
        std::vector<sd7_frame> fr = {frame(100, 64, 48), frame(100, 64, 48)};
        edit(fr[1]);
        expect_einval(what, fr, 2, cap);
    };
    bad("width 0", [](sd7_frame& f) { f.view.W = 0; });
    bad("height above the largest side", [](sd7_frame& f) { f.view.H = SD7_MAX_DIM + 1; });
    bad("focal length 0", [](sd7_frame& f) { f.view.fx = 0.0f; });
    bad("focal length NaN", [](sd7_frame& f) { f.view.fy = std::nanf(""); });
    bad("negative n", [](sd7_frame& f) { f.scene.n = -1; });
    bad("n of 2^31", [](sd7_frame& f) { f.scene.n = (int64_t)1 << 31; });
    bad("NULL scene array", [](sd7_frame& f) { f.scene.L = nullptr; });
    bad("NULL image", [](sd7_frame& f) { f.image = nullptr; });
    bad("NULL last", [](sd7_frame& f) { f.last = nullptr; });
    bad("negative pair capacity", [](sd7_frame&) {}, -1);
    bad("pair capacity of 2^31", [](sd7_frame&) {}, (int64_t)1 << 31);
    std::vector<sd7_frame> big(3, frame((int64_t)1 << 30, 64, 48));
    expect_einval("total Gaussians of 3 * 2^30", big, 3, 1024);
    std::printf("%d failed\n", failures);
    return failures;
}
