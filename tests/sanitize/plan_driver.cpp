// plan_driver.cpp -- exercises the host side of libsoft (plan tables, work
// lists and their checks, argument checks of every entry point) without a
// GPU, for a build of the library's host code with AddressSanitizer and
// UndefinedBehaviorSanitizer.  Exit status 0 when every call returns what
// include/soft.h documents and no sanitizer fires.
#include <cstdio>
#include <vector>

#include "soft.h"

static int bad = 0;
static void expect(int got, int want, const char *what) {
    if (got != want) {
        std::fprintf(stderr, "%s: %d, expected %d\n", what, got, want);
        bad = 1;
    }
}

int main() {
    // plan host sides: one bandwidth, batches, mixed bandwidths, every precision and flag
    const std::vector<std::vector<int>> cases = {
        {1}, {2}, {4}, {8}, {16}, {32}, {64}, {128}, {256}, {512}, {16, 16, 16},
        {1, 2, 4, 8, 16, 32, 64, 128}, {128, 4, 64, 4, 32, 1}, {512, 2, 256}, {1024}};
    for (const auto &bs : cases)
        for (int prec = 0; prec < 3; ++prec) {
            for (unsigned flags : {0u, 2u, 4u, 8u, 10u})
                expect(soft_plan_check(bs.data(), (int)bs.size(), prec, flags), SOFT_OK, "soft_plan_check");
            // the double-double recurrence: FP64 plans only
            for (unsigned flags : {16u, 26u})
                expect(soft_plan_check(bs.data(), (int)bs.size(), prec, flags), prec == 0 ? SOFT_OK : SOFT_ERR_INVALID,
                       "soft_plan_check dd");
        }
    std::vector<int> many(300);
    for (size_t i = 0; i < many.size(); ++i) many[i] = 1 << (i % 8);
    expect(soft_plan_check(many.data(), (int)many.size(), 2, 0), SOFT_OK, "300 functions");
    // argument errors
    const int odd[2] = {8, 12}, zero[2] = {8, 0}, big[1] = {2048};
    expect(soft_plan_check(nullptr, 1, 0, 0), SOFT_ERR_INVALID, "null list");
    expect(soft_plan_check(odd, 0, 0, 0), SOFT_ERR_INVALID, "n = 0");
    expect(soft_plan_check(zero, 2, 0, 0), SOFT_ERR_INVALID, "B = 0");
    expect(soft_plan_check(odd, 1, 3, 0), SOFT_ERR_INVALID, "precision");
    expect(soft_plan_check(odd, 1, 0, 32u), SOFT_ERR_INVALID, "flag");
    expect(soft_plan_check(odd, 2, 0, 0), SOFT_ERR_UNSUPPORTED, "B = 12");
    expect(soft_plan_check(big, 1, 0, 0), SOFT_ERR_UNSUPPORTED, "B = 2048");
    soft_plan_t h = nullptr;
    expect(soft_plan(0, 1, 0, 0, &h), SOFT_ERR_INVALID, "soft_plan B = 0");
    expect(soft_plan(8, 1, 0, 0, nullptr), SOFT_ERR_INVALID, "soft_plan out");
    expect(soft_plan_uneven(odd, 2, 0, 0, &h), SOFT_ERR_UNSUPPORTED, "soft_plan_uneven B = 12");
    expect(soft_forward(nullptr, nullptr, nullptr, nullptr), SOFT_ERR_INVALID, "soft_forward");
    expect(soft_plan_destroy(nullptr), SOFT_OK, "soft_plan_destroy");
    char buf[8];
    expect(soft_plan_describe(nullptr, buf, sizeof buf), SOFT_ERR_INVALID, "soft_plan_describe");
    expect(soft_match_argmax_noalloc(8, 0, 0, buf, nullptr, nullptr), SOFT_ERR_INVALID, "noalloc n = 0");
    expect(soft_probe_copy(buf, buf, 24, nullptr), SOFT_ERR_INVALID, "probe copy size");
    for (int s = 0; s >= -5; --s)
        if (!soft_status_string(s)) bad = 1;
    std::printf("plan host code under sanitizers: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
