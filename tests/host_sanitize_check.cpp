// Host code of the library under the address and undefined-behaviour
// sanitizers: the geometry and coefficient tables, the orbit builders and
// the binomial checkpoint schedule, over many inputs including edge cases
// and invalid ones.  Built with the host compiler and run by
// tests/test_host_sanitize.py; the device code is not involved.
#include <cmath>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "geometry.h"
#include "revolve.h"
#include "teuk.h"

namespace teuk_detail {
// the library's error helper (defined with the C ABI in capi.cpp)
thread_local std::string g_last_error;
int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}
}  // namespace teuk_detail

static long g_bad = 0;
#define EXPECT(cond)                                                           \
    do {                                                                       \
        if (!(cond)) {                                                         \
            ++g_bad;                                                           \
            std::printf("FAILED %s at line %d\n", #cond, __LINE__);            \
        }                                                                      \
    } while (0)

static bool all_finite(const std::vector<double>& v) {
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

static void geometry_cases() {
    struct G {
        double a;
        int s, m, nr, nth;
        double lo, hi;
    };
    const G grids[] = {{0.0, -2, 2, 801, 33, -100, 300},   {0.9, -2, 2, 6400, 128, -200, 600},
                       {0.99, -2, 4, 1600, 32, -200, 600}, {0.5, 2, 1, 5, 7, -50, 100},
                       {0.3, -2, 3, 12800, 256, -200, 600}, {0.7, 0, 0, 100, 9, -30, 60}};
    for (const auto& g : grids) {
        teuk::Geometry geo;
        const std::string err =
            teuk::build_geometry(1.0, g.a, g.s, g.m, g.nr, g.nth, g.lo, g.hi, 0.5, 0.5 * (g.lo + g.hi), geo);
        EXPECT(err.empty());
        EXPECT(all_finite(geo.rnode) && all_finite(geo.rhalf));
        EXPECT(static_cast<int>(geo.rows.size()) == g.nth);
        for (const auto& r : geo.rows) EXPECT(std::isfinite(r.cos_th) && std::isfinite(r.cot4h) && std::isfinite(r.V2));
        EXPECT(geo.dt > 0 && geo.i_ext >= 0 && geo.i_ext < g.nr);
    }
    // invalid descriptors come back as messages, not crashes
    teuk::Geometry geo;
    EXPECT(!teuk::build_geometry(1.0, 1.5, -2, 2, 100, 17, -50, 100, 0.5, 0, geo).empty());
    EXPECT(!teuk::build_geometry(1.0, 0.5, -2, 2, 2, 17, -50, 100, 0.5, 0, geo).empty());
    EXPECT(!teuk::build_geometry(1.0, 0.5, -2, 2, 100, 17, 100, -50, 0.5, 0, geo).empty());
    EXPECT(!teuk::build_geometry(1.0, 0.5, -2, 2, 100, 17, -50, 100, 0.5, 1e6, geo).empty());
    // the tortoise coordinate and its inverse
    for (double a : {0.0, 0.5, 0.9, 0.99})
        for (double x = 1e-6; x < 1e4; x *= 1.7) {
            const double rs = teuk::tortoise_of_x(x, 1.0, a);
            const double back = teuk::x_of_tortoise(rs, 1.0, a);
            EXPECT(std::fabs(back - x) <= 1e-9 * std::fmax(1.0, x));
        }
}

static void orbit_cases() {
    std::vector<double> out(3 * 2001);
    for (double a : {0.0, 0.3, 0.9, 0.99})
        for (double p : {6.0, 8.0, 10.0, 15.0})
            for (double e : {0.0, 0.1, 0.4, 0.7})
                for (double chi0 : {0.0, 1.3, 3.1}) {
                    const int rc = teuk_orbit_eccentric(1.0, a, p, e, chi0, 0.05, 2001, out.data());
                    if (rc == TEUK_OK)
                        EXPECT(all_finite(out));
                    else
                        EXPECT(rc == TEUK_EINVAL && !teuk_detail::g_last_error.empty());
                }
    EXPECT(teuk_orbit_eccentric(1.0, 0.5, 10.0, 0.95, 0.0, 0.05, 10, out.data()) == TEUK_EINVAL);
    EXPECT(teuk_orbit_eccentric(1.0, 1.5, 10.0, 0.2, 0.0, 0.05, 10, out.data()) == TEUK_EINVAL);
    EXPECT(teuk_orbit_eccentric(1.0, 0.5, 10.0, 0.2, 0.0, 0.05, -1, out.data()) == TEUK_EINVAL);
    EXPECT(teuk_orbit_eccentric(1.0, 0.5, 10.0, 0.2, 0.0, 0.05, 10, nullptr) == TEUK_EINVAL);
    EXPECT(teuk_orbit_eccentric(1.0, 0.5, 10.0, 0.2, 0.0, 0.05, 0, out.data()) == TEUK_OK);
}

static void schedule_cases() {
    for (int64_t n : {1, 2, 3, 7, 64, 100, 1000, 4096, 20000})
        for (int64_t s : {1, 2, 3, 5, 17, 64, 171, 5000}) {
            if (s == 1 && n > 1000) continue;   // quadratic recompute: valid, only slow
            teuk_detail::RevolveSchedule S;
            EXPECT(teuk_detail::revolve_schedule(n, s, &S));
            // replay on a symbolic state
            int64_t cur = 0, expect = n - 1, adv = 0;
            std::map<int64_t, int64_t> slots;
            for (const auto& a : S.forward) {
                if (a.op == teuk_detail::kStore) {
                    EXPECT(a.a >= 0 && a.a < s && a.b == cur);
                    slots[a.a] = cur;
                } else {
                    cur += a.a;
                    EXPECT(a.b == cur);
                }
            }
            EXPECT(cur == n);
            for (const auto& a : S.backward) {
                switch (a.op) {
                    case teuk_detail::kAdvance: cur += a.a; adv += a.a; EXPECT(a.b == cur); break;
                    case teuk_detail::kStore: EXPECT(a.a >= 0 && a.a < s && a.b == cur); slots[a.a] = cur; break;
                    case teuk_detail::kRestore: EXPECT(slots.count(a.a) && slots[a.a] == a.b); cur = a.b; break;
                    default: EXPECT(a.a == expect && cur == expect); --expect;
                }
            }
            EXPECT(expect == -1 && adv == S.backward_advances && S.slots_used <= s);
        }
    teuk_detail::RevolveSchedule S;
    EXPECT(!teuk_detail::revolve_schedule(0, 3, &S));
    EXPECT(!teuk_detail::revolve_schedule(10, 0, &S));
    EXPECT(teuk_detail::revolve_beta(3, 2) == 10);
    EXPECT(teuk_detail::revolve_beta(100000, 100000) == (int64_t(1) << 62));   // saturates, no overflow
}

int main() {
    geometry_cases();
    orbit_cases();
    schedule_cases();
    std::printf("host checks: %ld failed\n", g_bad);
    return g_bad != 0;
}
