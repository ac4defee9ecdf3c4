// Host-side check of the symmetric pair kernel's schedule arithmetic (SymSched, make_sym_sched):
// built with AddressSanitizer and UndefinedBehaviorSanitizer on the host side (the device code
// of pair.hip is compiled as usual and never launched) and run on the CPU by
// tests/test_native_sched.py.  For many sizes, widths and work-group counts: the super-block
// bases add up to the unit count, block_of inverts base, the work-group ranges begin(w) tile the
// units in order, wave_of inverts begin, the cost is monotone and ends at C, and the column
// partial count equals the symmetric units.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "common.hpp"

namespace tpe {
SymSched make_sym_sched(int64_t Fp, int W, int tail, int nw);
int64_t sym_colpart_floats(const SymSched& sc, bool grad);
}  // namespace tpe

using tpe::SymSched;

static int fails = 0;
#define CHECK(c, ...)                                                 \
    do {                                                              \
        if (!(c)) {                                                   \
            if (fails < 20) {                                         \
                std::printf("FAIL %s:%d: %s: ", __FILE__, __LINE__, #c); \
                std::printf(__VA_ARGS__);                             \
                std::printf("\n");                                    \
            }                                                         \
            ++fails;                                                  \
        }                                                             \
    } while (0)

static void check(int64_t nF, int nw, int W, int tail) {
    const int64_t sb = (int64_t)tpe::ROWB * nw;
    const int64_t Fp = (nF + sb - 1) / sb * sb;
    const SymSched s = tpe::make_sym_sched(Fp, W, tail, nw);
    CHECK(s.nw == nw && s.sbc == nw * tpe::ROWB / tpe::CHUNK, "nF %lld nw %d", (long long)nF, nw);
    CHECK(s.nsb == Fp / sb && s.nch == Fp / tpe::CHUNK, "nF %lld", (long long)nF);
    // units super block by super block: sbc diagonal units, then one per later chunk
    int64_t u = 0, sym = 0;
    for (int I = 0; I < s.nsb; ++I) {
        CHECK(s.base(I) == u, "base(%d) = %lld, expected %lld", I, (long long)s.base(I), (long long)u);
        CHECK(s.base_sym(I) == sym, "base_sym(%d)", I);
        const int64_t later = (int64_t)tpe::SUB * (s.nch - (int64_t)s.sbc * (I + 1));
        u += s.sbc + later;
        sym += later;
    }
    CHECK(s.U == u && s.base(s.nsb) == u, "U %lld vs %lld", (long long)s.U, (long long)u);
    CHECK(tpe::sym_colpart_floats(s, true) == sym * tpe::NSYM * tpe::SYM_COLS, "colpart");
    CHECK(tpe::sym_colpart_floats(s, false) == sym * tpe::SYM_COLS, "colpart energy");
    // block_of inverts base at the super-block boundaries and at sampled units
    std::vector<int64_t> us;
    for (int I = 0; I < s.nsb; I += 1 + s.nsb / 64) {
        us.push_back(s.base(I));
        if (s.base(I + 1) - 1 >= s.base(I)) us.push_back(s.base(I + 1) - 1);
    }
    for (int64_t k = 0; k < 200; ++k) us.push_back((s.U - 1) * k / 199);
    int64_t prev_cost = -1;
    for (int64_t x : us) {
        const int I = s.block_of(x);
        CHECK(I >= 0 && I < s.nsb && s.base(I) <= x && x < s.base(I + 1), "block_of(%lld) = %d", (long long)x, I);
    }
    for (int64_t k = 0; k <= 200; ++k) {
        const int64_t x = s.U * k / 200;
        const int64_t c = s.cost(x);
        CHECK(c >= prev_cost, "cost not monotone at %lld", (long long)x);
        prev_cost = c;
    }
    CHECK(s.cost(s.U) == s.C, "cost(U) %lld vs C %lld", (long long)s.cost(s.U), (long long)s.C);
    // the work-group ranges tile [0, U) in order, and wave_of finds the range of a unit
    CHECK(s.W >= 1 && s.W1 >= 1 && s.W1 <= s.W, "W %d W1 %d", s.W, s.W1);
    CHECK(s.begin(0) == 0 && s.begin(s.W) == s.U, "begin ends");
    const int step = s.W > 4096 ? s.W / 2048 : 1;
    int64_t last = 0;
    for (int w = 0; w <= s.W; w += step) {
        const int64_t b = s.begin(w);
        CHECK(b >= last && b <= s.U, "begin(%d) = %lld after %lld", w, (long long)b, (long long)last);
        last = b;
    }
    for (int64_t x : us) {
        const int w = s.wave_of(x);
        CHECK(w >= 0 && w < s.W && s.begin(w) <= x && x < s.begin(w + 1), "wave_of(%lld) = %d [%lld, %lld)",
              (long long)x, w, (long long)s.begin(w), (long long)s.begin(w + 1));
    }
}

int main() {
    int runs = 0;
    const int64_t sizes[] = {1, 20, 127, 128, 129, 320, 1280, 2001, 5000, 20480, 81920, 327680, 1310720};
    for (int nw : {1, 2, 4, 8})
        for (int64_t nF : sizes)
            for (int W : {1, 7, 1024, 4096, 32768})
                for (int tail : {0, 1, W}) {
                    check(nF, nw, W, tail);
                    ++runs;
                }
    std::printf("%d schedules checked, %d failures\n", runs, fails);
    return fails ? 1 : 0;
}
