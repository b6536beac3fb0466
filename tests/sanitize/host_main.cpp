// A driver of the library's host runtime for the AddressSanitizer / UBSan
// build (tests/test_sanitizers.py): descriptor validation (valid layouts,
// CFL and nesting violations, bad arguments, masked levels of touching
// blocks), the footprint, the fused kernel's tile plan at several tile
// heights, error strings, and the diagnostics' argument checks -- every path
// that runs without a GPU.
// Exit 0 when every call returns the expected code.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "rti.h"

extern "C" int rti_plan_tiles_for_test(const rti_domain_desc *desc, int th, int32_t *ntiles, int32_t *ndep,
                                       uint8_t *tinfo, uint8_t *tlev, int32_t *dep_off, int32_t *dep,
                                       uint32_t *tcmask);

static int failures = 0;
static void expect(int got, int want, const char *what)
{
    if (got != want) {
        std::fprintf(stderr, "%s: got %d, want %d (%s)\n", what, got, want, rti_last_error());
        ++failures;
    }
}

int main()
{
    const int nx0 = 60, ny0 = 48;
    std::vector<double> h0((size_t)nx0 * ny0), h1(36 * 27), h2(27 * 27);
    for (int j = 0; j < ny0; ++j)
        for (int i = 0; i < nx0; ++i) h0[(size_t)j * nx0 + i] = 200.0 - 4.0 * i;      // land in the east
    for (auto &v : h1) v = 40.0;
    for (auto &v : h2) v = 10.0;
    rti_level_desc lv[3] = {{nx0, ny0, -1, 0, 0, h0.data()}, {36, 27, 0, 20, 10, h1.data()},
                            {27, 27, 1, 3, 3, h2.data()}};
    rti_domain_desc d{};
    d.n_levels = 3;
    d.levels = lv;
    d.dx0 = 810.0;
    d.dt = 1.0;
    d.g = 9.81;
    d.manning_n = 0.025;
    d.dry_eps = 0.01;
    size_t bytes = 0;
    expect(rti_domain_footprint(&d, &bytes), RTI_OK, "footprint of a valid nest");
    if (bytes == 0) ++failures;
    for (int th : {4, 5, 12, 24, 64}) {
        int32_t nt = 0, nd = 0;
        expect(rti_plan_tiles_for_test(&d, th, &nt, &nd, nullptr, nullptr, nullptr, nullptr, nullptr), RTI_OK, "plan sizes");
        std::vector<uint8_t> tinfo(nt), tlev(nt);
        std::vector<int32_t> off(nt + 1), dep(nd > 0 ? nd : 1);
        std::vector<uint32_t> mask(nt);
        expect(rti_plan_tiles_for_test(&d, th, &nt, &nd, tinfo.data(), tlev.data(), off.data(), dep.data(), mask.data()),
               RTI_OK, "plan tables");
        for (int g = 0; g < nt; ++g)
            for (int k = off[g]; k < off[g + 1]; ++k)
                if (dep[k] < 0 || dep[k] >= nt) ++failures;
    }
    // the middle level as an L of two touching blocks (parent cells (6.., 5..) left out), its child
    // inside the L with 3 cells of margin, then a mask that is not constant over a 3x3 block
    std::vector<uint8_t> m1(36 * 27);
    for (int j = 0; j < 27; ++j)
        for (int i = 0; i < 36; ++i) m1[(size_t)j * 36 + i] = !(i >= 18 && j >= 15);
    lv[1].mask = m1.data();
    lv[2].nx = 9;
    lv[2].ny = 9;
    expect(rti_domain_footprint(&d, &bytes), RTI_OK, "footprint of a masked level");
    for (int th : {4, 7, 12}) {
        int32_t nt = 0, nd = 0;
        expect(rti_plan_tiles_for_test(&d, th, &nt, &nd, nullptr, nullptr, nullptr, nullptr, nullptr), RTI_OK,
               "masked plan sizes");
        std::vector<uint8_t> tinfo(nt), tlev(nt);
        std::vector<int32_t> off(nt + 1), dep(nd > 0 ? nd : 1);
        std::vector<uint32_t> mask(nt);
        expect(rti_plan_tiles_for_test(&d, th, &nt, &nd, tinfo.data(), tlev.data(), off.data(), dep.data(), mask.data()),
               RTI_OK, "masked plan tables");
    }
    lv[2].off_i = 14;                                    // the child's columns reach parent cell 16: 2 from the outside
    lv[2].off_j = 10;
    expect(rti_domain_footprint(&d, &bytes), RTI_ENEST, "child within 3 cells of a masked parent's outside");
    lv[2].off_i = 3;
    lv[2].off_j = 3;
    m1[5] = 0;                                           // one cell of a 3x3 block
    expect(rti_domain_footprint(&d, &bytes), RTI_ENEST, "mask not constant over a 3x3 block");
    lv[1].mask = nullptr;
    lv[2].nx = 27;
    lv[2].ny = 27;
    rti_domain_desc bad = d;
    lv[1].nx = 35;                                       // not a multiple of 3
    expect(rti_domain_footprint(&bad, &bytes), RTI_ENEST, "child nx not a multiple of 3");
    lv[1].nx = 36;
    lv[1].off_i = 1;                                     // margin below 3 parent cells
    expect(rti_domain_footprint(&bad, &bytes), RTI_ENEST, "child too close to the parent's edge");
    lv[1].off_i = 20;
    bad.dt = 10.0;                                       // CFL: 810 / 10 < sqrt(2 g 200)
    expect(rti_domain_footprint(&bad, &bytes), RTI_ECFL, "CFL violated");
    bad.dt = 1.0;
    bad.n_levels = 0;
    expect(rti_domain_footprint(&bad, &bytes), RTI_EINVAL, "no levels");
    bad.n_levels = 3;
    bad.precision = 7;
    expect(rti_domain_footprint(&bad, &bytes), RTI_EINVAL, "unknown precision");
    expect(rti_domain_footprint(nullptr, &bytes), RTI_EINVAL, "NULL descriptor");
    expect(rti_math_probe(9, nullptr, nullptr, 0, nullptr), RTI_EINVAL, "probe op");
    expect(rti_math_probe(RTI_PROBE_CBRT, nullptr, nullptr, 0, nullptr), RTI_OK, "empty probe");
    expect(rti_stream_probe(nullptr, 0, nullptr, 0, 0, nullptr), RTI_EINVAL, "stream probe reads");
    for (int c = 0; c >= -9; --c)
        if (!rti_strerror(c)) ++failures;
    rti_domain_destroy(nullptr);
    rti_batch_destroy(nullptr);
    if (failures) return 1;
    std::printf("host runtime ok\n");
    return 0;
}
