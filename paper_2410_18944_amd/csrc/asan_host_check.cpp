// Memory-error check of the host side of the C ABI: built from the host
// builder's source under AddressSanitizer and UndefinedBehaviorSanitizer
// (host code only; no device call is made), it runs wost_build_bvh on 2D and
// 3D scenes with mixed boundary conditions, open chains, duplicated and
// reversed primitives, every leaf size from 1 to 64 and the brute-force
// layout, queries the handles, and drives every rejection path (invalid
// dimensions, condition codes, vertex ids, non-finite vertices, degenerate
// primitives, NULL arguments, uploads without a buffer).  Exit status 0 and
// "asan host ok" on success.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../include/wost.h"

namespace {

int g_fail = 0;

void expect(bool ok, const char* what)
{
    if (!ok) {
        std::printf("FAILED: %s (%s)\n", what, wost_last_error());
        ++g_fail;
    }
}

struct Mesh {
    int dim;
    std::vector<float> v;
    std::vector<int32_t> p;
    std::vector<uint8_t> bc;
};

Mesh polygon(int n, bool open, unsigned seed)
{
    Mesh m{2, {}, {}, {}};
    for (int i = 0; i < n; ++i) {
        const double t = 2.0 * 3.14159265358979323846 * i / n;
        const double r = 1.0 + 0.2 * std::sin(7.0 * t + seed);
        m.v.push_back((float)(r * std::cos(t)));
        m.v.push_back((float)(r * std::sin(t)));
    }
    const int segs = open ? n - 1 : n;
    for (int i = 0; i < segs; ++i) {
        m.p.push_back(i);
        m.p.push_back((i + 1) % n);
        m.bc.push_back((uint8_t)(((i * 2654435761u + seed) >> 7) & 1u));
    }
    return m;
}

// latitude-longitude sphere, the northern half Neumann
Mesh sphere(int nlat, int nlon)
{
    Mesh m{3, {}, {}, {}};
    for (int a = 0; a <= nlat; ++a) {
        const double th = 3.14159265358979323846 * a / nlat;
        for (int b = 0; b < nlon; ++b) {
            const double ph = 2.0 * 3.14159265358979323846 * b / nlon;
            m.v.push_back((float)(std::sin(th) * std::cos(ph)));
            m.v.push_back((float)(std::sin(th) * std::sin(ph)));
            m.v.push_back((float)std::cos(th));
        }
    }
    auto id = [&](int a, int b) { return a * nlon + (b % nlon); };
    for (int a = 0; a < nlat; ++a) {
        for (int b = 0; b < nlon; ++b) {
            const int q[4] = {id(a, b), id(a + 1, b), id(a + 1, b + 1), id(a, b + 1)};
            const uint8_t c = a < nlat / 2 ? 1 : 0;
            if (a > 0) { m.p.insert(m.p.end(), {q[0], q[1], q[3]}); m.bc.push_back(c); }
            if (a + 1 < nlat) { m.p.insert(m.p.end(), {q[1], q[2], q[3]}); m.bc.push_back(c); }
        }
    }
    return m;
}

int build(const Mesh& m, int leaf, int brute, wost_geom** g)
{
    wost_build_opts o{leaf, brute};
    return wost_build_bvh(m.dim, m.v.data(), (int64_t)m.v.size() / m.dim, m.p.data(),
                          (int64_t)m.p.size() / m.dim, m.bc.data(), &o, g);
}

void check_valid(const Mesh& m, const char* name)
{
    const int64_t n = (int64_t)m.bc.size();
    for (int leaf : {1, 2, 4, 7, 16, 64}) {
        wost_geom* g = nullptr;
        expect(build(m, leaf, 0, &g) == WOST_OK && g, name);
        if (!g) continue;
        double info[8];
        expect(wost_geom_info(g, info) == WOST_OK, "info");
        expect(info[1] + info[2] == (double)n, "counts");
        expect(wost_geom_device_bytes(g) > 0 && wost_geom_device_bytes(g) % 256 == 0, "bytes");
        std::vector<int> seen(n, 0);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t c = wost_geom_prim_index(g, (int32_t)i);
            expect(c >= 0 && c < n, "prim index");
            if (c >= 0 && c < n) seen[c]++;
        }
        for (int64_t i = 0; i < n; ++i) expect(seen[i] == 1, "prim index is a permutation");
        expect(wost_geom_prim_index(g, (int32_t)n) == -1 && wost_geom_prim_index(g, -1) == -1, "index range");
        expect(wost_geom_upload(g, nullptr, 0, nullptr) == WOST_EINVAL, "upload without buffer");
        wost_geom_free(g);
    }
    wost_geom* g = nullptr;
    expect(build(m, 4, 1, &g) == WOST_OK && g, "brute force");
    wost_geom_free(g);
}

void check_rejections(const Mesh& m0)
{
    wost_geom* g = nullptr;
    Mesh m = m0;
    expect(wost_build_bvh(4, m.v.data(), 3, m.p.data(), 1, m.bc.data(), nullptr, &g) == WOST_EINVAL && !g, "dim");
    expect(wost_build_bvh(m.dim, m.v.data(), 3, m.p.data(), 1, m.bc.data(), nullptr, nullptr) == WOST_EINVAL, "out");
    expect(wost_build_bvh(m.dim, nullptr, 3, m.p.data(), 1, m.bc.data(), nullptr, &g) == WOST_EINVAL, "null verts");
    m.bc[1] = 3;
    expect(build(m, 4, 0, &g) == WOST_EINVAL && !g, "bc");
    m = m0;
    m.p[m.dim + 1] = (int32_t)(m.v.size() / m.dim);
    expect(build(m, 4, 0, &g) == WOST_EINVAL && !g, "vertex id");
    m = m0;
    m.p[1] = m.p[0];
    expect(build(m, 4, 0, &g) == WOST_EINVAL && !g, "degenerate");
    m = m0;
    m.v[0] = NAN;
    expect(build(m, 4, 0, &g) == WOST_EINVAL && !g, "non-finite");
    m = m0;
    expect(build(m, 0, 0, &g) == WOST_EINVAL && !g, "leaf 0");
    expect(build(m, 65, 0, &g) == WOST_EINVAL && !g, "leaf 65");
    wost_geom_free(nullptr);
    double info[8];
    expect(wost_geom_info(nullptr, info) == WOST_EINVAL, "info of NULL");
    expect(wost_geom_device_bytes(nullptr) == -1, "bytes of NULL");
}

}  // namespace

int main()
{
    Mesh a = polygon(257, false, 1), b = polygon(64, true, 2), c = sphere(24, 32);
    // duplicated and reversed segments
    Mesh d = polygon(40, false, 3);
    for (int i = 0; i < 8; ++i) {
        d.p.push_back(d.p[2 * i + 1]);
        d.p.push_back(d.p[2 * i]);
        d.bc.push_back(1);
    }
    check_valid(a, "2D closed polygon");
    check_valid(b, "2D open chain");
    check_valid(c, "3D sphere");
    check_valid(d, "2D duplicated and reversed segments");
    check_rejections(a);
    check_rejections(c);
    if (g_fail) {
        std::printf("asan host check: %d failures\n", g_fail);
        return 1;
    }
    std::printf("asan host ok\n");
    return 0;
}
