// Sanitizer driver (CPU only): the host side of libnsa (validation, block pattern, colouring, every
// tile plan, the scalar CSR view, error paths) and the C oracle (pattern, assembly, row assembly,
// explicit residual) on meshes read from files, built with AddressSanitizer and
// UndefinedBehaviorSanitizer. It checks the library's pattern against the oracle's and touches every
// index a plan hands to a kernel; the sanitizers check every access on the way.
//
// Mesh file: int64 npoin, int64 nelem, then int32 lnods[nelem][4], double coord[npoin][3],
// double velocity[npoin][3].
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "nsa.h"

extern "C" {
int64_t oracle_pattern(int64_t npoin, int64_t nelem, const int32_t *lnods, int64_t *bptr, int32_t *bcol,
                       int32_t *emap);
int oracle_assemble(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord, const double *veloc,
                    double rho, double mu, double dt, int64_t nnzb, const int32_t *emap, double *values, double *rhs);
int oracle_assemble_rows(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord,
                         const double *veloc, double rho, double mu, double dt, int64_t nsample,
                         const int64_t *rowslot, int32_t maxdeg, int32_t *cols, int32_t *deg, double *vals,
                         double *rhs_s);
int oracle_residual(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord, const double *veloc,
                    double rho, double mu, double dt, double *rhsid, double *dt_rho, double *mass_rho);
int oracle_validate(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord, int64_t *bad);
}

static int failures = 0;
#define CHECK(cond, ...)                                 \
    do {                                                 \
        if (!(cond)) {                                   \
            std::fprintf(stderr, "CHECK failed: " __VA_ARGS__); \
            std::fprintf(stderr, " (%s:%d)\n", __FILE__, __LINE__); \
            failures++;                                  \
        }                                                \
    } while (0)

struct Mesh {
    int64_t npoin = 0, nelem = 0;
    std::vector<int32_t> lnods;
    std::vector<double> coord, vel;
};

static bool read_mesh(const char *path, Mesh &m) {
    FILE *f = std::fopen(path, "rb");
    if (!f) return false;
    bool ok = std::fread(&m.npoin, 8, 1, f) == 1 && std::fread(&m.nelem, 8, 1, f) == 1;
    if (ok) {
        m.lnods.resize(4 * m.nelem);
        m.coord.resize(3 * m.npoin);
        m.vel.resize(3 * m.npoin);
        ok = std::fread(m.lnods.data(), 4, m.lnods.size(), f) == m.lnods.size() &&
             std::fread(m.coord.data(), 8, m.coord.size(), f) == m.coord.size() &&
             std::fread(m.vel.data(), 8, m.vel.size(), f) == m.vel.size();
    }
    std::fclose(f);
    return ok;
}

// every array a tiled plan hands to the kernel, read back and bounds-checked
static void check_tiles(nsa_mesh *h, const Mesh &m, int scatter) {
    nsa_mesh_info info;
    CHECK(nsa_mesh_get_info(h, &info) == NSA_OK, "info");
    const int64_t nt = info.ntiles[scatter], nr = info.tile_runs[scatter];
    if (!nt) return;
    std::vector<int32_t> row(nt + 1), relems(4 * nr);
    std::vector<int64_t> rptr(nt + 1), nptr(nt + 1);
    std::vector<uint8_t> runs(32 * nr);
    CHECK(nsa_mesh_get_tiles(h, scatter, nullptr, nullptr, nullptr, nptr.data(), nullptr, nullptr) == NSA_OK, "tiles");
    std::vector<int32_t> nodes(nptr[nt]);
    CHECK(nsa_mesh_get_tiles(h, scatter, row.data(), rptr.data(), relems.data(), nptr.data(), nodes.data(),
                             runs.data()) == NSA_OK, "tiles");
    std::vector<int64_t> bptr(m.npoin + 1);
    CHECK(nsa_mesh_get_pattern(h, bptr.data(), nullptr, nullptr) == NSA_OK, "pattern");
    int64_t pairs = 0;
    for (int64_t t = 0; t < nt; t++) {
        const int64_t nrows = row[t + 1] - row[t], nnod = nptr[t + 1] - nptr[t];
        const int64_t nblk = bptr[row[t + 1]] - bptr[row[t]];
        for (int64_t q = rptr[t]; q < rptr[t + 1]; q++) {
            uint16_t f[16];
            std::memcpy(f, runs.data() + 32 * q, 32);
            const int len = f[3];
            CHECK(len >= 1 && len <= 4 && f[0] < nrows && f[1] < nnod && f[2] < nnod, "run %lld header", (long long)q);
            CHECK(f[4] < nblk && f[5] < nblk && f[6] < nblk && f[7] == 0, "run %lld slots", (long long)q);
            for (int e = 0; e < len; e++) {
                CHECK(f[8 + e] < nnod && f[12 + e] < nblk, "run %lld element %d", (long long)q, e);
                const int32_t el = relems[4 * q + e];
                CHECK(el >= 0 && el < m.nelem, "run %lld element id", (long long)q);
            }
            pairs += len;
        }
    }
    CHECK(pairs == 4 * m.nelem, "pairs %lld != 4 nelem", (long long)pairs);
}

static void exercise(const Mesh &m) {
    const int32_t *ln = m.lnods.data();
    // standalone pattern against the oracle's
    std::vector<int64_t> bptr(m.npoin + 1), obptr(m.npoin + 1);
    int64_t nnzb = -1;
    CHECK(nsa_pattern_count(m.npoin, m.nelem, ln, bptr.data(), &nnzb) == NSA_OK, "count");
    std::vector<int32_t> bcol(nnzb > 0 ? nnzb : 1), emap(16 * m.nelem), ocol(16 * m.nelem + 1), oemap(16 * m.nelem);
    CHECK(nsa_pattern_fill(m.npoin, m.nelem, ln, bptr.data(), bcol.data(), emap.data()) == NSA_OK, "fill");
    const int64_t onnzb = oracle_pattern(m.npoin, m.nelem, ln, obptr.data(), ocol.data(), oemap.data());
    CHECK(onnzb == nnzb && bptr == obptr && std::equal(bcol.begin(), bcol.begin() + nnzb, ocol.begin()) && emap == oemap,
          "library pattern != oracle pattern");
    // oracle routes
    std::vector<double> values(16 * (nnzb > 0 ? nnzb : 1)), rhs(4 * m.npoin), rid(3 * m.npoin), dtr(m.npoin), mr(m.npoin);
    CHECK(oracle_assemble(m.npoin, m.nelem, ln, m.coord.data(), m.vel.data(), 1.0, 1e-3, 1e-2, nnzb, oemap.data(),
                          values.data(), rhs.data()) == 0, "oracle assemble");
    CHECK(oracle_residual(m.npoin, m.nelem, ln, m.coord.data(), m.vel.data(), 1.0, 1e-3, 1e-2, rid.data(),
                          dtr.data(), mr.data()) == 0, "oracle residual");
    {
        int32_t maxdeg = 0;
        for (int64_t i = 0; i < m.npoin; i++) maxdeg = std::max<int32_t>(maxdeg, (int32_t)(bptr[i + 1] - bptr[i]));
        std::vector<int64_t> slot(m.npoin, -1);
        int64_t ns = 0;
        for (int64_t i = 0; i < m.npoin; i += 3) slot[i] = ns++;
        std::vector<int32_t> cols(ns * maxdeg + 1), deg(ns + 1);
        std::vector<double> vals(16 * ns * maxdeg + 1), rs(4 * ns + 1);
        CHECK(oracle_assemble_rows(m.npoin, m.nelem, ln, m.coord.data(), m.vel.data(), 1.0, 1e-3, 1e-2, ns, slot.data(),
                                   maxdeg, cols.data(), deg.data(), vals.data(), rs.data()) == 0, "oracle rows");
        int64_t bad = 0;
        CHECK(oracle_validate(m.npoin, m.nelem, ln, m.coord.data(), &bad) == 0, "validate");
    }
    // a registered mesh with every plan at several sizes
    const int32_t sizes[][5] = {{64, 64, 64, 1, 64}, {512, 160, 512, 16, 128}, {1024, 1024, 4096, 256, 192},
                                {200, 96, 320, 64, 256}};
    for (const auto &sz : sizes) {
        nsa_mesh *h = nullptr;
        CHECK(nsa_mesh_create(m.npoin, m.nelem, ln, m.coord.data(), &h) == NSA_OK, "create: %s", nsa_last_error());
        if (!h) return;
        CHECK(nsa_mesh_set_tiling(h, NSA_ATOMIC, sz[0]) == NSA_OK, "tiling");
        CHECK(nsa_mesh_set_tiling(h, NSA_COLOUR, sz[1]) == NSA_OK, "tiling");
        CHECK(nsa_mesh_set_tiling(h, NSA_GATHER_PLAN, sz[2]) == NSA_OK, "tiling");
        CHECK(nsa_mesh_set_tiling(h, NSA_RESIDUAL_PLAN, sz[3]) == NSA_OK, "tiling");
        CHECK(nsa_mesh_set_tile_threads(h, sz[4]) == NSA_OK, "threads");
        nsa_mesh_info info;
        CHECK(nsa_mesh_get_info(h, &info) == NSA_OK, "info: %s", nsa_last_error());
        check_tiles(h, m, NSA_ATOMIC);
        check_tiles(h, m, NSA_COLOUR);
        if (info.gather_ntiles) {
            const int64_t gt = info.gather_ntiles, gr = info.gather_records, gp = info.gather_pairs;
            std::vector<int32_t> row(gt + 1), elems(gr);
            std::vector<int64_t> nptr(gt + 1), eptr(gt + 1), pptr(gt + 1);
            std::vector<uint16_t> loc(4 * gr), pairs(gp);
            std::vector<uint32_t> slots(m.npoin ? info.nnzb : 1);
            CHECK(nsa_mesh_get_gather(h, nullptr, nptr.data(), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                      nullptr) == NSA_OK, "gather");
            std::vector<int32_t> nodes(nptr[gt]);
            CHECK(nsa_mesh_get_gather(h, row.data(), nptr.data(), nodes.data(), eptr.data(), elems.data(), loc.data(),
                                      pptr.data(), pairs.data(), slots.data()) == NSA_OK, "gather");
        }
        if (info.residual_ntiles) {
            const int64_t rt = info.residual_ntiles, rr = info.residual_records;
            std::vector<int32_t> row(rt + 1), elems(rr);
            std::vector<int64_t> eptr(rt + 1), nptr(rt + 1);
            std::vector<uint16_t> loc(4 * rr);
            CHECK(nsa_mesh_get_residual_tiles(h, nullptr, nullptr, nullptr, nullptr, nptr.data(), nullptr) == NSA_OK, "res");
            std::vector<int32_t> nodes(nptr[rt]);
            CHECK(nsa_mesh_get_residual_tiles(h, row.data(), eptr.data(), elems.data(), loc.data(), nptr.data(),
                                              nodes.data()) == NSA_OK, "res");
        }
        std::vector<int64_t> rp(4 * m.npoin + 1);
        std::vector<int32_t> sc(16 * info.nnzb + 1);
        CHECK(nsa_pattern_scalar_csr(h, rp.data(), sc.data()) == NSA_OK, "scalar csr");
        std::vector<int32_t> cptr(info.ncolours + 1), celems(m.nelem + 1);
        CHECK(nsa_mesh_get_colouring(h, cptr.data(), celems.data()) == NSA_OK, "colouring");
        // calls out of order or with bad arguments are refused without touching anything
        CHECK(nsa_assemble(h, nullptr, 1, 1, 1, nullptr, nullptr, nullptr, nullptr) == NSA_ESTATE, "assemble before upload");
        CHECK(nsa_mesh_set_tile_threads(h, 96) == NSA_EINVAL, "bad threads");
        CHECK(nsa_mesh_set_tiling(h, 7, 64) == NSA_EINVAL, "bad plan");
        CHECK(nsa_mesh_release_host(h) == NSA_ESTATE, "release before upload");
        CHECK(nsa_mesh_destroy(h) == NSA_OK, "destroy");
    }
    // validation errors
    if (m.nelem > 1) {
        std::vector<int32_t> bad(m.lnods);
        bad[4 * (m.nelem - 1) + 2] = (int32_t)m.npoin;
        nsa_mesh *h = nullptr;
        CHECK(nsa_mesh_create(m.npoin, m.nelem, bad.data(), m.coord.data(), &h) == NSA_ERANGE && !h, "ERANGE");
        std::vector<double> flat(m.coord);
        for (int a = 1; a < 4; a++)
            for (int d = 0; d < 3; d++) flat[3 * m.lnods[a] + d] = flat[3 * m.lnods[0] + d];
        CHECK(nsa_mesh_create(m.npoin, m.nelem, m.lnods.data(), flat.data(), &h) == NSA_EDEGENERATE && !h, "EDEGENERATE");
    }
}

// Quadrilateral meshes: an n x n grid of the unit square with every node moved a little (seeded), its
// nodes relabelled by a fixed permutation; create, both row-tile plans, every record's indices.
void exercise_q1(int n, int tile_blocks) {
    const int64_t np = (int64_t)(n + 1) * (n + 1), ne = (int64_t)n * n;
    std::vector<int64_t> perm((size_t)np);
    for (int64_t i = 0; i < np; i++) perm[(size_t)i] = (i * 7919) % np;  // a bijection: 7919 is prime, np < 7919^2
    bool bij = true;
    {
        std::vector<char> hit((size_t)np, 0);
        for (int64_t i = 0; i < np; i++) hit[(size_t)perm[(size_t)i]]++;
        for (char c : hit) bij = bij && c == 1;
    }
    if (!bij)
        for (int64_t i = 0; i < np; i++) perm[(size_t)i] = i;
    std::vector<double> coord(2 * (size_t)np);
    uint64_t z = 12345;
    for (int j = 0; j <= n; j++)
        for (int i = 0; i <= n; i++) {
            const int64_t id = perm[(size_t)(i + (n + 1) * j)];
            z = z * 6364136223846793005ull + 1442695040888963407ull;
            const double jx = ((double)(z >> 11) * 0x1.0p-53 - 0.5) * 0.3 / n;
            z = z * 6364136223846793005ull + 1442695040888963407ull;
            const double jy = ((double)(z >> 11) * 0x1.0p-53 - 0.5) * 0.3 / n;
            coord[2 * id] = (double)i / n + jx;
            coord[2 * id + 1] = (double)j / n + jy;
        }
    std::vector<int32_t> ln(4 * (size_t)ne);
    for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) {
            const int64_t e = i + (int64_t)n * j;
            const int64_t v[4] = {i + (int64_t)(n + 1) * j, i + 1 + (int64_t)(n + 1) * j, i + 1 + (int64_t)(n + 1) * (j + 1),
                                  i + (int64_t)(n + 1) * (j + 1)};
            for (int a = 0; a < 4; a++) ln[4 * e + a] = (int32_t)perm[(size_t)v[a]];
        }
    nsa_mesh *h = nullptr;
    CHECK(nsa_mesh_create_q1(np, ne, ln.data(), coord.data(), &h) == NSA_OK, "q1 create: %s", nsa_last_error());
    if (!h) return;
    CHECK(nsa_mesh_set_tiling(h, NSA_ATOMIC, tile_blocks) == NSA_OK, "q1 tiling");
    nsa_mesh_info info;
    CHECK(nsa_mesh_get_info(h, &info) == NSA_OK && info.family == NSA_QUAD4, "q1 info");
    std::vector<int64_t> bptr((size_t)np + 1);
    std::vector<int32_t> bcol((size_t)info.nnzb), emap(16 * (size_t)ne);
    CHECK(nsa_mesh_get_pattern(h, bptr.data(), bcol.data(), emap.data()) == NSA_OK, "q1 pattern");
    for (int sc = 0; sc < 2; sc++) {
        const int64_t nt = info.ntiles[sc], nr = info.tile_runs[sc];
        std::vector<int32_t> row((size_t)nt + 1), elems((size_t)nr);
        std::vector<int64_t> eptr((size_t)nt + 1), nptr((size_t)nt + 1);
        std::vector<uint16_t> recs(24 * (size_t)nr);
        CHECK(nsa_mesh_get_q1_tiles(h, sc, nullptr, nullptr, nullptr, nullptr, nptr.data(), nullptr) == NSA_OK, "q1 nptr");
        std::vector<int32_t> nodes((size_t)nptr[(size_t)nt]);
        CHECK(nsa_mesh_get_q1_tiles(h, sc, row.data(), eptr.data(), elems.data(), recs.data(), nptr.data(), nodes.data()) ==
                  NSA_OK, "q1 tiles");
        for (int64_t t = 0; t < nt; t++) {
            const int64_t nblk = bptr[(size_t)row[(size_t)t + 1]] - bptr[(size_t)row[(size_t)t]];
            const int64_t nnod = nptr[(size_t)t + 1] - nptr[(size_t)t];
            for (int64_t p = eptr[(size_t)t]; p < eptr[(size_t)t + 1]; p++) {
                const uint16_t *r = &recs[24 * (size_t)p];
                for (int a = 0; a < 4; a++) {
                    CHECK(r[a] < nnod, "q1 local id");
                    CHECK(nodes[(size_t)(nptr[(size_t)t] + r[a])] == ln[4 * (size_t)elems[(size_t)p] + a], "q1 node");
                    if ((r[4] >> a) & 1)
                        for (int b = 0; b < 4; b++) CHECK(r[6 + 4 * a + b] < nblk, "q1 slot");
                }
            }
        }
    }
    nsa_mesh_destroy(h);
}

int main(int argc, char **argv) {
    exercise_q1(1, 64);
    exercise_q1(17, 64);
    exercise_q1(40, 768);
    std::printf("quadrilateral meshes done\n");
    for (int k = 1; k < argc; k++) {
        Mesh m;
        if (!read_mesh(argv[k], m)) {
            std::fprintf(stderr, "cannot read %s\n", argv[k]);
            return 2;
        }
        exercise(m);
        std::printf("%s: npoin %lld nelem %lld done\n", argv[k], (long long)m.npoin, (long long)m.nelem);
    }
    std::printf("failures %d\n", failures);
    return failures ? 1 : 0;
}
