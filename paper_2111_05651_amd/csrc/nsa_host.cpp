// Host side of libnsa: argument checking, validation, the block pattern of the node graph,
// element colouring, the device data layout and the dispatch of the assembly kernels.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <unordered_map>

#include "nsa_internal.h"

namespace {

// Message of the calling thread's last failed call (a fixed buffer: recording an error allocates nothing).
thread_local char g_last_error[512];

nsa_status fail(nsa_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return st;
}

nsa_status ok() {
    g_last_error[0] = '\0';
    return NSA_OK;
}

int host_threads() {
    unsigned n = std::thread::hardware_concurrency();
    if (n == 0) n = 1;
    return (int)std::min(16u, n);
}

// Run f(begin, end) over [0, n) split into contiguous chunks on up to host_threads() threads.
template <class F>
void parallel_for(int64_t n, F f, int64_t grain = 4096) {
    int nt = host_threads();
    if (n < grain * 2 || nt == 1) {
        f(int64_t(0), n);
        return;
    }
    nt = (int)std::min<int64_t>(nt, (n + grain - 1) / grain);
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (int t = 0; t < nt; t++) {
        int64_t b = t * chunk, e = std::min(n, b + chunk);
        if (b >= e) break;
        th.emplace_back([=] { f(b, e); });
    }
    for (auto &t : th) t.join();
}

// Node -> element adjacency (counting sort by node): elements of node i are
// list[ptr[i] .. ptr[i+1]), ascending.
void node_elements(int64_t npoin, int64_t nelem, const int32_t *lnods, std::vector<int64_t> &ptr,
                   std::vector<int32_t> &list) {
    ptr.assign(npoin + 1, 0);
    for (int64_t e = 0; e < nelem; e++)
        for (int a = 0; a < 4; a++) ptr[lnods[4 * e + a] + 1]++;
    for (int64_t i = 0; i < npoin; i++) ptr[i + 1] += ptr[i];
    list.resize(ptr[npoin]);
    std::vector<int64_t> pos(ptr.begin(), ptr.end() - 1);
    for (int64_t e = 0; e < nelem; e++)
        for (int a = 0; a < 4; a++) list[pos[lnods[4 * e + a]]++] = (int32_t)e;
}

nsa_status check_range(int64_t npoin, int64_t nelem, const int32_t *lnods) {
    std::atomic<int64_t> bad{-1};
    parallel_for(nelem, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; i++)
            for (int a = 0; a < 4; a++) {
                int32_t v = lnods[4 * i + a];
                if (v < 0 || v >= npoin) {
                    int64_t cur = bad.load();
                    while ((cur < 0 || i < cur) && !bad.compare_exchange_weak(cur, i)) {
                    }
                }
            }
    });
    if (bad.load() >= 0)
        return fail(NSA_ERANGE, "element %lld has a node id outside [0, %lld)", (long long)bad.load(),
                    (long long)npoin);
    return NSA_OK;
}

// Row degrees from the node-element adjacency: the distinct nodes of the elements around node i.
nsa_status pattern_rows(int64_t npoin, const int32_t *lnods, const std::vector<int64_t> &n2e_ptr,
                        const std::vector<int32_t> &n2e, std::vector<int64_t> &bptr,
                        std::vector<int32_t> *bcol) {
    if (!bcol) bptr.assign(npoin + 1, 0);
    parallel_for(npoin, [&](int64_t b, int64_t e) {
        std::vector<int32_t> cand;
        for (int64_t i = b; i < e; i++) {
            cand.clear();
            for (int64_t k = n2e_ptr[i]; k < n2e_ptr[i + 1]; k++) {
                const int32_t *en = lnods + 4 * (int64_t)n2e[k];
                cand.insert(cand.end(), en, en + 4);
            }
            std::sort(cand.begin(), cand.end());
            auto last = std::unique(cand.begin(), cand.end());
            int64_t deg = last - cand.begin();
            if (!bcol)
                bptr[i + 1] = deg;
            else
                std::copy(cand.begin(), last, bcol->begin() + bptr[i]);
        }
    }, 1024);
    if (!bcol)
        for (int64_t i = 0; i < npoin; i++) bptr[i + 1] += bptr[i];
    return NSA_OK;
}

void fill_emap(int64_t nelem, const int32_t *lnods, const int64_t *bptr, const int32_t *bcol,
               int32_t *emap) {
    parallel_for(nelem, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; i++)
            for (int a = 0; a < 4; a++) {
                int32_t row = lnods[4 * i + a];
                const int32_t *lo = bcol + bptr[row], *hi = bcol + bptr[row + 1];
                for (int c = 0; c < 4; c++) {
                    const int32_t *p = std::lower_bound(lo, hi, lnods[4 * i + c]);
                    emap[16 * i + 4 * a + c] = (int32_t)(p - bcol);
                }
            }
    });
}

// Jacobian determinant of the affine map of element e (columns X_{s+1} - X_0).
double elem_det(const int32_t *ln, const double *coord) {
    double J[3][3];
    const double *x0 = coord + 3 * (int64_t)ln[0];
    for (int s = 0; s < 3; s++) {
        const double *xs = coord + 3 * (int64_t)ln[s + 1];
        for (int r = 0; r < 3; r++) J[r][s] = xs[r] - x0[r];
    }
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// Greedy first-fit colouring in element order with per-node colour masks (up to 128 colours).
nsa_status colour_elements(nsa_mesh *m) {
    const int64_t n = m->nelem;
    // colours 0..127 of every node in two inline words; colours from 128 on (nodes in more than
    // 128 elements) in per-node overflow bitsets
    std::vector<uint64_t> mask(2 * (size_t)m->npoin, 0);
    std::unordered_map<int32_t, std::vector<uint64_t>> extra;
    std::vector<int32_t> col(n);
    int32_t ncol = 0;
    for (int64_t e = 0; e < n; e++) {
        uint64_t f0 = 0, f1 = 0;
        const int32_t *ln = &m->lnods[4 * e];
        for (int a = 0; a < 4; a++) {
            f0 |= mask[2 * (size_t)ln[a]];
            f1 |= mask[2 * (size_t)ln[a] + 1];
        }
        int c;
        if (~f0) {
            c = __builtin_ctzll(~f0);
        } else if (~f1) {
            c = 64 + __builtin_ctzll(~f1);
        } else {
            size_t words = 0;
            for (int a = 0; a < 4; a++) {
                auto it = extra.find(ln[a]);
                if (it != extra.end()) words = std::max(words, it->second.size());
            }
            c = -1;
            for (size_t w = 0; w <= words && c < 0; w++) {
                uint64_t f = 0;
                for (int a = 0; a < 4; a++) {
                    auto it = extra.find(ln[a]);
                    if (it != extra.end() && w < it->second.size()) f |= it->second[w];
                }
                if (~f) c = 128 + 64 * (int)w + __builtin_ctzll(~f);
            }
        }
        for (int a = 0; a < 4; a++) {
            if (c < 128) {
                mask[2 * (size_t)ln[a] + (c >> 6)] |= 1ull << (c & 63);
            } else {
                std::vector<uint64_t> &x = extra[ln[a]];
                const size_t w = (size_t)(c - 128) >> 6;
                if (x.size() <= w) x.resize(w + 1, 0);
                x[w] |= 1ull << ((c - 128) & 63);
            }
        }
        col[e] = c;
        ncol = std::max(ncol, c + 1);
    }
    m->ncolours = ncol;
    m->colour_ptr.assign(ncol + 1, 0);
    for (int64_t e = 0; e < n; e++) m->colour_ptr[col[e] + 1]++;
    for (int c = 0; c < ncol; c++) m->colour_ptr[c + 1] += m->colour_ptr[c];
    m->colour_elems.resize(n);
    std::vector<int32_t> pos(m->colour_ptr.begin(), m->colour_ptr.end() - 1);
    for (int64_t e = 0; e < n; e++) m->colour_elems[pos[col[e]]++] = (int32_t)e;
    return NSA_OK;
}

// Default tile plans: the throughput plan uses 512-block tiles (80 KB of LDS, two workgroups of
// four wavefronts per CU); the deterministic plan uses 128-block tiles (20 KB, eight one-wavefront
// workgroups per CU, as many as the registers allow; larger tiles hold fewer wavefronts, smaller ones
// evaluate more elements twice. 128^3: 1.546 / 1.434 ms FP64 / mixed against 1.563 / 1.535 at 160).
constexpr int32_t kDefaultTileBlocks[2] = {512, 128};
constexpr int32_t kPlanThreads[2] = {256, 64};
constexpr int32_t kMaxTileBlocks = 1024;
constexpr int32_t kMaxTileRows = 256;
constexpr int64_t kMaxTileLds = 160 * 1024;  // LDS one workgroup may use on gfx950

// Run f(chunk, begin, end) over [0, n) in up to host_threads() contiguous chunks; returns the
// number of chunks used.
template <class F>
int parallel_chunks(int64_t n, F f) {
    int nt = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), n / 64));
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    int used = 0;
    for (int t = 0; t < nt; t++) {
        int64_t b = t * chunk, e = std::min(n, b + chunk);
        if (b >= e) break;
        used++;
        th.emplace_back([=] { f(t, b, e); });
    }
    for (auto &t : th) t.join();
    return used;
}

// Record order of a tile: groups of 16 consecutive records (the lanes whose 8-byte LDS atomics
// the LDS serves together: 16 lanes over 32 four-byte banks) chosen so that, for each owned-row
// iteration k and column b, the blocks the lanes add into sit on different bank pairs (value i of
// block slot s of the tile lies on bank pair (17 s + i) mod 16) and in different rows (same row:
// same diagonal block, same address). Each record may take its owned rows in any order and its
// other vertices in any order; the chosen vertex order is written back to vord. Records stay grouped
// by owned-row count; each slot of a group takes, among the next 8 records of the count, the one (and
// vertex order) that adds the least to the lanes already placed in the group.
// by_row: the adds of owned-row iteration k go to per-row accumulators (the residual tiles: double
// 5 r + c of the tile's accumulators, bank pair (5 r + c) mod 16), so the bank pair of a lane follows
// its row alone and only the order of the owned rows matters.
void bank_order(const nsa_mesh *m, const std::vector<int32_t> &els, const std::vector<int32_t> &nown, int32_t r0,
                bool by_row, const std::vector<int32_t> &base, std::vector<int8_t> &vord, std::vector<int32_t> &out) {
    constexpr int kWindow = 8;
    const size_t ne = base.size();
    out.clear();
    out.reserve(ne);
    const int64_t b0 = m->bptr[r0];
    constexpr int kGroup = 16;
    uint8_t cnt[4][4][kGroup], peak[4][4];
    uint32_t rows[4][2];  // rows used per iteration k (local rows < 64 tracked, others ignored)
    int fill = kGroup;
    // all vertex orders of a record: owned part permuted, then the other part permuted
    auto orders = [&](int32_t j, int8_t (*cand)[4]) -> int {
        int8_t o[4], x[4];
        const int n = nown[j];
        for (int q = 0; q < 4; q++) (q < n ? o[q] : x[q - n]) = vord[4 * j + q];
        std::sort(o, o + n);
        std::sort(x, x + 4 - n);
        int c = 0;
        do {
            int8_t xx[4];
            std::copy(x, x + 4 - n, xx);
            do {
                if (c == 24) return c;
                for (int q = 0; q < n; q++) cand[c][q] = o[q];
                for (int q = n; q < 4; q++) cand[c][q] = xx[q - n];
                c++;
            } while (!by_row && std::next_permutation(xx, xx + 4 - n));
        } while (std::next_permutation(o, o + n));
        return c;
    };
    // cost of placing record j with vertex order v: a row already used by iteration k (same diagonal
    // block), then for each (k, b) the lanes already on that bank pair, heavily if the record would
    // raise the instruction's worst bank pair (the LDS needs one pass per lane on that pair)
    auto cost = [&](int32_t j, const int8_t *v) -> int {
        const int64_t e = els[j];
        const int32_t *ln = &m->lnods[4 * e];
        int c = 0;
        for (int k = 0; k < nown[j]; k++) {
            const int lr = ln[v[k]] - r0;
            if (lr < 64 && ((rows[k][lr >> 5] >> (lr & 31)) & 1u)) c += 64;
            for (int b = 0; b < 4; b++) {
                const int64_t slot = by_row ? 5 * lr : m->emap[16 * e + 4 * v[k] + v[b]] - b0;
                const int n = cnt[k][b][slot & (kGroup - 1)];
                c += n >= peak[k][b] ? 16 * (n + 1) : n;
            }
        }
        return c;
    };
    auto place = [&](int32_t j, const int8_t *v) {
        const int64_t e = els[j];
        const int32_t *ln = &m->lnods[4 * e];
        for (int k = 0; k < nown[j]; k++) {
            const int lr = ln[v[k]] - r0;
            if (lr < 64) rows[k][lr >> 5] |= 1u << (lr & 31);
            for (int b = 0; b < 4; b++) {
                const int64_t slot = by_row ? 5 * lr : m->emap[16 * e + 4 * v[k] + v[b]] - b0;
                const int n = ++cnt[k][b][slot & (kGroup - 1)];
                peak[k][b] = std::max<int>(peak[k][b], n);
            }
        }
        for (int q = 0; q < 4; q++) vord[4 * j + q] = v[q];
        out.push_back(j);
        fill++;
    };
    std::vector<int32_t> pool;
    int8_t cand[24][4];
    size_t g0 = 0;
    while (g0 < ne) {
        size_t g1 = g0;
        while (g1 < ne && nown[base[g1]] == nown[base[g0]]) g1++;
        pool.assign(base.begin() + g0, base.begin() + g1);
        g0 = g1;
        size_t head = 0;  // pool[head ..] remain, in base order
        while (head < pool.size()) {
            if (fill == kGroup) {
                std::memset(cnt, 0, sizeof(cnt));
                std::memset(peak, 0, sizeof(peak));
                std::memset(rows, 0, sizeof(rows));
                fill = 0;
            }
            size_t best = head;
            int bestc = 1 << 30;
            int8_t bestv[4] = {0, 1, 2, 3};
            for (size_t q = head; q < pool.size() && q < head + kWindow; q++) {
                const int nc = orders(pool[q], cand);
                for (int c = 0; c < nc; c++) {
                    const int v = cost(pool[q], cand[c]);
                    if (v < bestc) {
                        bestc = v;
                        best = q;
                        std::copy(cand[c], cand[c] + 4, bestv);
                    }
                }
                if (!bestc) break;
            }
            place(pool[best], bestv);
            std::swap(pool[best], pool[head]);
            head++;
        }
    }
}

// ---- run plan of the tiled kernel ------------------------------------------------------------

// A run in global node ids (see nsa::RunRec): row i, hinge j, k_old of its first element, and per
// element its id and k_new.
struct GRun {
    int32_t row, hinge, k0, len;
    int32_t el[nsa::kRunMax], knew[nsa::kRunMax];
};

// Partition the elements around node i (star[0 .. ns)) into runs of at most kRunMax elements. The
// elements that contain both i and a node j form the ring of the edge (i, j); two of them are
// neighbours in the ring when they share a face (i, j, k). Greedy: among all hinges j, walk the
// longest chain of still unassigned ring neighbours (cut at kRunMax), preferring a chain that is
// complete within kRunMax (the ring of a face-diagonal edge of a Kuhn cube has four elements, and
// those six rings partition the 24 elements around an interior node), then the shortest complete
// chain; take it as one run and repeat. Any chain is correct; the choice only sets how many runs a
// row needs (each run costs one set of register sums to add into the tile image).
void row_runs(const nsa_mesh *m, int32_t i, const int32_t *star, int64_t ns, std::vector<GRun> &out) {
    struct El {
        int32_t e, v[3];  // element and its three vertices other than i
        bool used;
    };
    std::vector<El> els((size_t)ns);
    std::vector<int32_t> hinges;
    for (int64_t q = 0; q < ns; q++) {
        const int32_t *ln = &m->lnods[4 * (int64_t)star[q]];
        El &x = els[(size_t)q];
        x.e = star[q];
        x.used = false;
        int c = 0;
        for (int a = 0; a < 4; a++)
            if (ln[a] != i && c < 3) x.v[c++] = ln[a];
        hinges.insert(hinges.end(), x.v, x.v + 3);
    }
    std::sort(hinges.begin(), hinges.end());
    hinges.erase(std::unique(hinges.begin(), hinges.end()), hinges.end());
    // the two vertices of element x other than i and j (j is one of x.v)
    auto others = [](const El &x, int32_t j, int32_t &a, int32_t &b) {
        int c = 0;
        int32_t o[2] = {-1, -1};
        for (int q = 0; q < 3; q++)
            if (x.v[q] != j && c < 2) o[c++] = x.v[q];
        a = o[0];
        b = o[1];
    };
    auto has = [](const El &x, int32_t g) { return x.v[0] == g || x.v[1] == g || x.v[2] == g; };
    std::vector<int32_t> ring, chain, kn, best_chain, best_kn;
    std::vector<char> seen;
    int64_t left = ns;
    while (left > 0) {
        int32_t best_j = -1, best_k0 = -1;
        int best_take = 0, best_full = 0;
        bool best_fits = false;
        for (int32_t j : hinges) {
            ring.clear();
            for (size_t q = 0; q < els.size(); q++)
                if (!els[q].used && has(els[q], j)) ring.push_back((int32_t)q);
            if (ring.empty()) continue;
            const size_t rn = ring.size();
            // ring neighbours share a vertex besides i and j; walk every chain once, from an end
            // (an element with at most one neighbour) or, for a closed ring, from any element
            std::vector<int32_t> ka(rn), kb(rn), deg(rn, 0);
            for (size_t q = 0; q < rn; q++) others(els[(size_t)ring[q]], j, ka[q], kb[q]);
            for (size_t q = 0; q < rn; q++)
                for (size_t p = 0; p < rn; p++)
                    if (p != q && (ka[p] == ka[q] || ka[p] == kb[q] || kb[p] == ka[q] || kb[p] == kb[q])) deg[q]++;
            seen.assign(rn, 0);
            for (int pass = 0; pass < 2; pass++) {
                for (size_t s0 = 0; s0 < rn; s0++) {
                    if (seen[s0] || (pass == 0 && deg[s0] > 1)) continue;
                    // leave the start through a vertex it shares with a neighbour, if any
                    int32_t k0 = ka[s0], k1 = kb[s0];
                    bool out_b = false;
                    for (size_t p = 0; p < rn && !out_b; p++)
                        if (p != s0 && (ka[p] == kb[s0] || kb[p] == kb[s0])) out_b = true;
                    if (!out_b) std::swap(k0, k1);
                    chain.assign(1, (int32_t)s0);
                    kn.assign(1, k1);
                    seen[s0] = 1;
                    int32_t kcur = k1;
                    while (true) {
                        size_t nx = rn;
                        for (size_t p = 0; p < rn; p++)
                            if (!seen[p] && (ka[p] == kcur || kb[p] == kcur)) {
                                nx = p;
                                break;
                            }
                        if (nx == rn) break;
                        const int32_t knext = ka[nx] == kcur ? kb[nx] : ka[nx];
                        seen[nx] = 1;
                        chain.push_back((int32_t)nx);
                        kn.push_back(knext);
                        kcur = knext;
                    }
                    const int full = (int)chain.size();
                    const int take = std::min(full, nsa::kRunMax);
                    const bool fits = full <= nsa::kRunMax;
                    const bool better = take > best_take || (take == best_take && fits && !best_fits) ||
                                        (take == best_take && fits == best_fits && full < best_full);
                    if (better) {
                        best_take = take;
                        best_full = full;
                        best_fits = fits;
                        best_j = j;
                        best_k0 = k0;
                        best_chain.clear();
                        for (int q = 0; q < take; q++) best_chain.push_back(ring[(size_t)chain[(size_t)q]]);
                        best_kn.assign(kn.begin(), kn.begin() + take);
                    }
                }
            }
        }
        GRun r{};
        r.row = i;
        r.hinge = best_j;
        r.k0 = best_k0;
        r.len = best_take;
        for (int q = 0; q < nsa::kRunMax; q++) {
            r.el[q] = q < best_take ? els[(size_t)best_chain[(size_t)q]].e : -1;
            r.knew[q] = q < best_take ? best_kn[(size_t)q] : -1;
        }
        for (int q = 0; q < best_take; q++) els[(size_t)best_chain[(size_t)q]].used = true;
        left -= best_take;
        out.push_back(r);
    }
}

// Order of the runs of a tile (their lanes): length descending, so that the lanes of a wavefront
// walk runs of the same length; inside each wavefront's 64 runs, groups of 16 consecutive runs (the lanes whose
// 8-byte LDS atomics the LDS serves together: 16 lanes over 32 four-byte banks) chosen greedily so
// that the runs of a group belong to different rows (same row: the same diagonal block, RHS row and
// possibly the same (i, k) blocks, i.e. the same addresses, which the LDS serialises) and that, for
// every add instruction, their target slots fall on different bank pairs (value v of slot s lies on
// bank pair (s + v) mod 16 with the 17-double slot stride; RHS row r on (5 r + c) mod 16).
void run_order(const std::vector<nsa::RunRec> &runs, std::vector<int32_t> &order) {
    constexpr int kGroup = 16, kWave = 64, kTypes = nsa::kRunMax + 4;
    const size_t n = runs.size();
    // start from the rows interleaved (the first run of every row, then the second, ...), so that a
    // window of consecutive candidates spans many rows
    std::vector<int32_t> base(n), ordinal(n);
    {
        std::unordered_map<int, int> seen;
        for (size_t q = 0; q < n; q++) ordinal[q] = seen[runs[q].row]++;
    }
    for (size_t q = 0; q < n; q++) base[q] = (int32_t)q;
    std::stable_sort(base.begin(), base.end(), [&](int32_t x, int32_t y) {
        if (runs[x].len != runs[y].len) return runs[x].len > runs[y].len;
        if (ordinal[x] != ordinal[y]) return ordinal[x] < ordinal[y];
        return runs[x].row < runs[y].row;
    });
    order.clear();
    order.reserve(n);
    uint8_t cnt[kTypes][kGroup];
    std::vector<int32_t> rows;
    int fill = kGroup;
    auto slot_of = [&](const nsa::RunRec &r, int t) -> int {
        if (t < nsa::kRunMax) return t < r.len ? r.kslot[t] : -1;
        switch (t - nsa::kRunMax) {
            case 0: return r.last;
            case 1: return r.jslot;
            case 2: return r.diag;
            default: return 5 * r.row;
        }
    };
    auto cost = [&](const nsa::RunRec &r) -> int {
        int c = 256 * (int)std::count(rows.begin(), rows.end(), (int32_t)r.row);
        for (int t = 0; t < kTypes; t++) {
            const int s = slot_of(r, t);
            if (s >= 0) c += cnt[t][s & (kGroup - 1)];
        }
        return c;
    };
    size_t head = 0;
    while (head < n) {
        if (fill == kGroup) {
            std::memset(cnt, 0, sizeof cnt);
            rows.clear();
            fill = 0;
        }
        size_t best = head;
        int bestc = 1 << 30;
        const size_t wave_end = std::min(n, (head / kWave + 1) * kWave);
        for (size_t q = head; q < wave_end; q++) {
            const int c = cost(runs[base[q]]);
            if (c < bestc) {
                bestc = c;
                best = q;
            }
            if (!c) break;
        }
        const nsa::RunRec &r = runs[base[best]];
        for (int t = 0; t < kTypes; t++) {
            const int s = slot_of(r, t);
            if (s >= 0) cnt[t][s & (kGroup - 1)]++;
        }
        rows.push_back(r.row);
        order.push_back(base[best]);
        std::swap(base[best], base[head]);  // inside one wavefront's 64 runs
        head++;
        fill++;
    }
}

// Nodes that row r adds to the node list of tile `tid`: the row node itself (an owned row is in its
// tile's node list even when no element touches it, so it has no diagonal block) and the columns of
// its blocks not yet in the list.
int64_t row_new_nodes(const nsa_mesh *m, const std::vector<int32_t> &stamp, int64_t r, int32_t tid) {
    int64_t add = stamp[(size_t)r] != tid;
    for (int64_t k = m->bptr[r]; k < m->bptr[r + 1]; k++) {
        const int32_t c = m->bcol[k];
        add += c != r && stamp[(size_t)c] != tid;
    }
    return add;
}

void stamp_row(const nsa_mesh *m, std::vector<int32_t> &stamp, int64_t r, int32_t tid) {
    stamp[(size_t)r] = tid;
    for (int64_t k = m->bptr[r]; k < m->bptr[r + 1]; k++) stamp[(size_t)m->bcol[k]] = tid;
}

// Row tiles for the tiled kernel (see nsa_internal.h). A tile is a contiguous row range whose LDS
// footprint (block image, RHS rows, node table) stays within tile_blocks * 160 bytes and whose runs
// number at most threads - 64 (threads for a one-wavefront workgroup): one run per lane, a single
// row with more runs takes several rounds.
// Per tile: the nodes its elements touch (the owned rows first, as local ids 0 .. nrows-1, then the
// other nodes ascending) and the runs of its rows in the order of run_order().
nsa_status build_tiles(nsa_mesh *m, nsa::TilePlan &P, int32_t tile_blocks, int32_t threads) {
    P = nsa::TilePlan();
    P.tile_blocks = tile_blocks;
    P.threads = threads;
    // uint16 slots and local node ids bound what the tiled kernel can address
    if (m->max_row_blocks > 256 || m->npoin == 0) return NSA_OK;
    const int64_t np = m->npoin;
    const int64_t one_row = (int64_t)nsa::tile_lds_bytes((int32_t)m->max_row_blocks, 1, (int32_t)m->max_row_blocks);
    if (one_row > kMaxTileLds) return NSA_OK;  // a single row would not fit in LDS
    const int64_t budget = std::max<int64_t>(std::min<int64_t>((int64_t)tile_blocks * 160, kMaxTileLds), one_row);
    std::vector<int64_t> n2e_ptr;
    std::vector<int32_t> n2e;
    node_elements(np, m->nelem, m->lnods.data(), n2e_ptr, n2e);
    // runs of every row (independent of the tiling)
    std::vector<std::vector<GRun>> rr((size_t)host_threads());
    std::vector<int64_t> row_nruns((size_t)np + 1, 0);
    {
        const int nth = host_threads();
        const int64_t chunk = (np + nth - 1) / nth;
        std::vector<std::thread> th;
        for (int c = 0; c < nth; c++) {
            const int64_t b = c * chunk, e = std::min<int64_t>(np, b + chunk);
            if (b >= e) continue;
            th.emplace_back([&, c, b, e] {
                for (int64_t i = b; i < e; i++) {
                    const size_t before = rr[(size_t)c].size();
                    row_runs(m, (int32_t)i, n2e.data() + n2e_ptr[i], n2e_ptr[i + 1] - n2e_ptr[i], rr[(size_t)c]);
                    row_nruns[(size_t)i + 1] = (int64_t)(rr[(size_t)c].size() - before);
                }
            });
        }
        for (auto &t : th) t.join();
    }
    for (int64_t i = 0; i < np; i++) row_nruns[(size_t)i + 1] += row_nruns[(size_t)i];
    std::vector<GRun> allruns;
    allruns.reserve((size_t)row_nruns[(size_t)np]);
    for (auto &v : rr) {
        allruns.insert(allruns.end(), v.begin(), v.end());
        std::vector<GRun>().swap(v);
    }
    // grow tiles row by row; the touched nodes of a tile are the columns of its rows
    // runs per tile: one per lane of all but the last wavefront of a multi-wavefront workgroup, which
    // takes part only in the prologue and the write-out (with every wavefront holding runs, the last
    // one was mostly empty at the LDS budget's tile size and still issued the full element code; as a
    // helper it speeds up the memory phases: 128^3, 512-block tiles, 256 threads, FP64 / mixed
    // 1.71 / 1.58 ms with runs on all four wavefronts, 1.64 / 1.49 ms with three)
    const int64_t run_cap = threads > 64 ? threads - 64 : threads;
    std::vector<int32_t> stamp(np, -1);
    P.row.push_back(0);
    int32_t tid = 0;
    for (int64_t r0 = 0; r0 < np; tid++) {
        int64_t r1 = r0, nodes = 0;
        while (r1 < np) {
            const int64_t add = row_new_nodes(m, stamp, r1, tid);
            const int64_t blocks = m->bptr[r1 + 1] - m->bptr[r0];
            const int64_t need = (int64_t)nsa::tile_lds_bytes((int32_t)blocks, (int32_t)(r1 + 1 - r0), (int32_t)(nodes + add));
            const int64_t nruns = row_nruns[(size_t)r1 + 1] - row_nruns[(size_t)r0];
            if (r1 > r0 && (need > budget || r1 + 1 - r0 > kMaxTileRows || nruns > run_cap)) break;
            stamp_row(m, stamp, r1, tid);
            nodes += add;
            r1++;
        }
        if (nodes > 65535) return fail(NSA_EUNSUPPORTED, "a tile touches more than 65535 nodes");
        P.row.push_back((int32_t)r1);
        P.cap_rows = std::max<int32_t>(P.cap_rows, (int32_t)(r1 - r0));
        P.cap_blocks = std::max<int32_t>(P.cap_blocks, (int32_t)(m->bptr[r1] - m->bptr[r0]));
        P.cap_nodes = std::max<int32_t>(P.cap_nodes, (int32_t)nodes);
        P.cap_runs = std::max<int32_t>(P.cap_runs, (int32_t)(row_nruns[(size_t)r1] - row_nruns[(size_t)r0]));
        P.lds = std::max<int64_t>(P.lds, (int64_t)nsa::tile_lds_bytes((int32_t)(m->bptr[r1] - m->bptr[r0]),
                                                                      (int32_t)(r1 - r0), (int32_t)nodes));
        r0 = r1;
    }
    std::vector<int32_t>().swap(stamp);
    const int64_t nt = (int64_t)P.row.size() - 1;
    struct Out {
        std::vector<int32_t> nodes, relems;
        std::vector<nsa::RunRec> runs;
        std::vector<int64_t> cnt, ncnt;
        int64_t pairs = 0;
    };
    std::vector<Out> outs(host_threads());
    int used = parallel_chunks(nt, [&](int ci, int64_t tb, int64_t te) {
        Out &o = outs[ci];
        std::vector<int32_t> other, order;
        std::vector<nsa::RunRec> loc;
        std::vector<int32_t> locel;
        for (int64_t t = tb; t < te; t++) {
            const int32_t r0 = P.row[t], r1 = P.row[t + 1], nr = r1 - r0;
            const int64_t b0 = m->bptr[r0];
            // node table: owned rows, then the other touched nodes (columns of the rows) ascending
            other.clear();
            for (int32_t i = r0; i < r1; i++)
                for (int64_t k = m->bptr[i]; k < m->bptr[i + 1]; k++)
                    if (m->bcol[k] < r0 || m->bcol[k] >= r1) other.push_back(m->bcol[k]);
            std::sort(other.begin(), other.end());
            other.erase(std::unique(other.begin(), other.end()), other.end());
            for (int32_t i = r0; i < r1; i++) o.nodes.push_back(i);
            o.nodes.insert(o.nodes.end(), other.begin(), other.end());
            o.ncnt.push_back((int64_t)nr + (int64_t)other.size());
            auto local = [&](int32_t g) -> uint16_t {
                if (g >= r0 && g < r1) return (uint16_t)(g - r0);
                return (uint16_t)(nr + (std::lower_bound(other.begin(), other.end(), g) - other.begin()));
            };
            auto slot = [&](int32_t i, int32_t g) -> uint16_t {
                const int32_t *lo = m->bcol.data() + m->bptr[i], *hi = m->bcol.data() + m->bptr[i + 1];
                return (uint16_t)(m->bptr[i] - b0 + (std::lower_bound(lo, hi, g) - lo));
            };
            loc.clear();
            locel.clear();
            for (int64_t q = row_nruns[(size_t)r0]; q < row_nruns[(size_t)r1]; q++) {
                const GRun &g = allruns[(size_t)q];
                nsa::RunRec r{};
                r.row = (uint16_t)(g.row - r0);
                r.hinge = local(g.hinge);
                r.k0 = local(g.k0);
                r.len = (uint16_t)g.len;
                r.diag = slot(g.row, g.row);
                r.jslot = slot(g.row, g.hinge);
                r.last = slot(g.row, g.knew[g.len - 1]);
                for (int e = 0; e < nsa::kRunMax; e++) {
                    r.knew[e] = e < g.len ? local(g.knew[e]) : 0;
                    r.kslot[e] = e < g.len ? slot(g.row, e == 0 ? g.k0 : g.knew[e - 1]) : 0;
                    locel.push_back(g.el[e]);
                }
                o.pairs += g.len;
                loc.push_back(r);
            }
            run_order(loc, order);
            for (int32_t q : order) {
                o.runs.push_back(loc[(size_t)q]);
                o.relems.insert(o.relems.end(), locel.begin() + nsa::kRunMax * q, locel.begin() + nsa::kRunMax * (q + 1));
            }
            o.cnt.push_back((int64_t)loc.size());
        }
    });
    std::vector<GRun>().swap(allruns);
    P.rptr.assign(1, 0);
    P.nptr.assign(1, 0);
    for (int i = 0; i < used; i++) {
        Out &o = outs[i];
        for (size_t k = 0; k < o.cnt.size(); k++) {
            P.rptr.push_back(P.rptr.back() + o.cnt[k]);
            P.nptr.push_back(P.nptr.back() + o.ncnt[k]);
        }
        P.nodes.insert(P.nodes.end(), o.nodes.begin(), o.nodes.end());
        P.runs.insert(P.runs.end(), o.runs.begin(), o.runs.end());
        P.relems.insert(P.relems.end(), o.relems.begin(), o.relems.end());
        P.npairs += o.pairs;
        o = Out();
    }
    if ((int64_t)P.rptr.size() != nt + 1 || P.npairs != 4 * m->nelem)
        return fail(NSA_EUNSUPPORTED, "tile plan inconsistent");
    P.ok = true;
    return NSA_OK;
}

// Gather tiles (see nsa_internal.h): contiguous row ranges grown while the tile stays within
// tile_blocks blocks, 4095 elements, 65535 contributions, 80 KB of LDS in the mixed form (two
// workgroups per CU) and 160 KB with FP64 element data. Records are the elements
// touching the tile in ascending element id with the local ids of their vertices; every block's
// contributions follow in record order; slots order the blocks by contribution count, descending.
constexpr int32_t kGatherThreads = 256;
constexpr int32_t kMaxGatherBlocks = 4096;
constexpr int32_t kMaxGatherRecs = 4095;
constexpr int64_t kMaxGatherPairs = 65535;
constexpr int64_t kGatherLdsMixed = 80 * 1024;  // two workgroups per CU in the mixed form

nsa_status build_gather(nsa_mesh *m, nsa::GatherPlan &P, int32_t tile_blocks, int32_t threads) {
    P = nsa::GatherPlan();
    P.tile_blocks = tile_blocks;
    P.threads = threads;
    const int64_t np = m->npoin;
    if (np == 0) return NSA_OK;
    std::vector<int64_t> n2e_ptr;
    std::vector<int32_t> n2e;
    node_elements(np, m->nelem, m->lnods.data(), n2e_ptr, n2e);
    std::vector<int32_t> stamp(np, -1), estamp(m->nelem, -1);
    P.row.push_back(0);
    int32_t tid = 0;
    for (int64_t r0 = 0; r0 < np; tid++) {
        int64_t r1 = r0, nodes = 0, recs = 0, pairs = 0;
        while (r1 < np) {
            const int64_t addn = row_new_nodes(m, stamp, r1, tid);
            int64_t adde = 0;
            for (int64_t k = n2e_ptr[r1]; k < n2e_ptr[r1 + 1]; k++) adde += estamp[n2e[k]] != tid;
            const int64_t addp = 4 * (n2e_ptr[r1 + 1] - n2e_ptr[r1]);
            const int64_t blocks = m->bptr[r1 + 1] - m->bptr[r0];
            const int32_t nn = (int32_t)(nodes + addn), nre = (int32_t)(recs + adde), npa = (int32_t)(pairs + addp);
            const int64_t lds = nsa::gather_lds_bytes(nn, nre, npa, true);
            const int64_t lds32 = nsa::gather_lds_bytes(nn, nre, npa, false);
            const bool over = blocks > tile_blocks || lds > kMaxTileLds || lds32 > kGatherLdsMixed ||
                              recs + adde > kMaxGatherRecs ||
                              pairs + addp > kMaxGatherPairs || nodes + addn > 65535;
            if (over && r1 > r0) break;
            if (over) return NSA_OK;  // one row alone does not fit: no gather plan for this mesh
            stamp_row(m, stamp, r1, tid);
            for (int64_t k = n2e_ptr[r1]; k < n2e_ptr[r1 + 1]; k++) estamp[n2e[k]] = tid;
            nodes += addn;
            recs += adde;
            pairs += addp;
            r1++;
        }
        P.row.push_back((int32_t)r1);
        r0 = r1;
    }
    std::vector<int32_t>().swap(stamp);
    std::vector<int32_t>().swap(estamp);
    const int64_t nt = (int64_t)P.row.size() - 1;
    P.slots.assign(m->nnzb, 0);
    struct Out {
        std::vector<int32_t> els, nodes;
        std::vector<uint2> recs;
        std::vector<uint16_t> pairs;
        std::vector<int64_t> ecnt, ncnt, pcnt;
        int32_t cap_blocks = 0, cap_recs = 0, cap_nodes = 0, cap_pairs = 0;
        int64_t lds64 = 0, lds32 = 0;
    };
    std::vector<Out> outs(host_threads());
    int used = parallel_chunks(nt, [&](int ci, int64_t tb, int64_t te) {
        Out &o = outs[ci];
        std::vector<int32_t> els, other, cnt, order, start, fill;
        std::vector<uint32_t> tmp;  // (record << 4 | a << 2 | b) per contribution, grouped by block
        for (int64_t t = tb; t < te; t++) {
            const int32_t r0 = P.row[t], r1 = P.row[t + 1], nr = r1 - r0;
            const int64_t b0 = m->bptr[r0];
            const int32_t nb = (int32_t)(m->bptr[r1] - b0);
            els.clear();
            for (int32_t i = r0; i < r1; i++) els.insert(els.end(), n2e.begin() + n2e_ptr[i], n2e.begin() + n2e_ptr[i + 1]);
            std::sort(els.begin(), els.end());
            els.erase(std::unique(els.begin(), els.end()), els.end());
            other.clear();
            for (int32_t e : els)
                for (int a = 0; a < 4; a++) {
                    const int32_t g = m->lnods[4 * (int64_t)e + a];
                    if (g < r0 || g >= r1) other.push_back(g);
                }
            std::sort(other.begin(), other.end());
            other.erase(std::unique(other.begin(), other.end()), other.end());
            for (int32_t i = r0; i < r1; i++) o.nodes.push_back(i);
            o.nodes.insert(o.nodes.end(), other.begin(), other.end());
            const int32_t nnod = nr + (int32_t)other.size();
            auto local = [&](int32_t g) -> uint32_t {
                if (g >= r0 && g < r1) return (uint32_t)(g - r0);
                return (uint32_t)(nr + (std::lower_bound(other.begin(), other.end(), g) - other.begin()));
            };
            // contributions per block, in record order
            cnt.assign(nb, 0);
            for (size_t ri = 0; ri < els.size(); ri++) {
                const int64_t e = els[ri];
                for (int a = 0; a < 4; a++) {
                    const int32_t g = m->lnods[4 * e + a];
                    if (g < r0 || g >= r1) continue;
                    for (int b = 0; b < 4; b++) cnt[m->emap[16 * e + 4 * a + b] - b0]++;
                }
            }
            start.assign(nb + 1, 0);
            for (int32_t k = 0; k < nb; k++) start[k + 1] = start[k] + cnt[k];
            const int32_t npair = start[nb];
            tmp.assign(npair, 0);
            fill.assign(start.begin(), start.end() - 1);
            for (size_t ri = 0; ri < els.size(); ri++) {
                const int64_t e = els[ri];
                const int32_t *ln = &m->lnods[4 * e];
                o.recs.push_back(make_uint2(local(ln[0]) | local(ln[1]) << 16, local(ln[2]) | local(ln[3]) << 16));
                o.els.push_back((int32_t)e);
                for (int a = 0; a < 4; a++) {
                    if (ln[a] < r0 || ln[a] >= r1) continue;
                    for (int b = 0; b < 4; b++)
                        tmp[fill[m->emap[16 * e + 4 * a + b] - b0]++] = (uint32_t)ri << 4 | (uint32_t)a << 2 | (uint32_t)b;
                }
            }
            // slots: longest lists first, then block order
            order.resize(nb);
            for (int32_t k = 0; k < nb; k++) order[k] = k;
            std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cnt[x] > cnt[y]; });
            int32_t off = 0;
            for (int32_t sidx = 0; sidx < nb; sidx++) {
                const int32_t k = order[sidx];
                P.slots[b0 + sidx] = (uint32_t)k << 16 | (uint32_t)off;
                for (int32_t q = start[k]; q < start[k + 1]; q++) o.pairs.push_back((uint16_t)tmp[q]);
                off += cnt[k];
            }
            o.ecnt.push_back((int64_t)els.size());
            o.ncnt.push_back(nnod);
            o.pcnt.push_back(npair);
            o.cap_blocks = std::max(o.cap_blocks, nb);
            o.cap_recs = std::max(o.cap_recs, (int32_t)els.size());
            o.cap_nodes = std::max(o.cap_nodes, nnod);
            o.cap_pairs = std::max(o.cap_pairs, npair);
            o.lds64 = std::max(o.lds64, nsa::gather_lds_bytes(nnod, (int32_t)els.size(), npair, true));
            o.lds32 = std::max(o.lds32, nsa::gather_lds_bytes(nnod, (int32_t)els.size(), npair, false));
        }
    });
    P.eptr.assign(1, 0);
    P.nptr.assign(1, 0);
    P.pptr.assign(1, 0);
    for (int i = 0; i < used; i++) {
        Out &o = outs[i];
        for (size_t k = 0; k < o.ecnt.size(); k++) {
            P.eptr.push_back(P.eptr.back() + o.ecnt[k]);
            P.nptr.push_back(P.nptr.back() + o.ncnt[k]);
            P.pptr.push_back(P.pptr.back() + o.pcnt[k]);
        }
        P.elems.insert(P.elems.end(), o.els.begin(), o.els.end());
        P.nodes.insert(P.nodes.end(), o.nodes.begin(), o.nodes.end());
        P.recs.insert(P.recs.end(), o.recs.begin(), o.recs.end());
        P.pairs.insert(P.pairs.end(), o.pairs.begin(), o.pairs.end());
        P.cap_blocks = std::max(P.cap_blocks, o.cap_blocks);
        P.cap_recs = std::max(P.cap_recs, o.cap_recs);
        P.cap_nodes = std::max(P.cap_nodes, o.cap_nodes);
        P.cap_pairs = std::max(P.cap_pairs, o.cap_pairs);
        P.lds[0] = std::max(P.lds[0], o.lds64);
        P.lds[1] = std::max(P.lds[1], o.lds32);
        o = Out();
    }
    if ((int64_t)P.eptr.size() != nt + 1) return fail(NSA_EUNSUPPORTED, "gather plan inconsistent");
    P.ok = true;
    return NSA_OK;
}

// Residual tiles (see nsa_internal.h): contiguous row ranges of at most tile_rows rows whose LDS
// (48 bytes per touched node, 40 per owned row) stays within kResLds (two workgroups per CU or
// more). Records: the elements touching the tile, local node ids owned nodes first, ordered by
// owned-node count (descending; the lanes of a wavefront run the same number of row iterations),
// then by bank_order() with per-row accumulators: the 16 lanes of a group add into rows distinct
// mod 16 where the tile allows it, so their five accumulator adds touch distinct bank pairs.
constexpr int64_t kResLds = 64 * 1024;
constexpr int32_t kMaxResRows = 4096;

nsa_status build_rtiles(nsa_mesh *m, nsa::ResPlan &P, int32_t tile_rows) {
    P = nsa::ResPlan();
    P.tile_rows = tile_rows;
    const int64_t np = m->npoin;
    if (np == 0) return NSA_OK;
    if (nsa::res_lds_bytes((int32_t)m->max_row_blocks, 1) > kResLds) return NSA_OK;
    std::vector<int32_t> stamp(np, -1);
    P.row.push_back(0);
    int32_t tid = 0;
    for (int64_t r0 = 0; r0 < np; tid++) {
        int64_t r1 = r0, nodes = 0;
        while (r1 < np) {
            const int64_t add = row_new_nodes(m, stamp, r1, tid);
            const int64_t need = nsa::res_lds_bytes((int32_t)(nodes + add), (int32_t)(r1 + 1 - r0));
            if (r1 > r0 && (need > kResLds || r1 + 1 - r0 > tile_rows || nodes + add > 65535)) break;
            stamp_row(m, stamp, r1, tid);
            nodes += add;
            r1++;
        }
        P.row.push_back((int32_t)r1);
        P.lds = std::max<int64_t>(P.lds, nsa::res_lds_bytes((int32_t)nodes, (int32_t)(r1 - r0)));
        r0 = r1;
    }
    std::vector<int32_t>().swap(stamp);
    const int64_t nt = (int64_t)P.row.size() - 1;
    std::vector<int64_t> n2e_ptr;
    std::vector<int32_t> n2e;
    node_elements(np, m->nelem, m->lnods.data(), n2e_ptr, n2e);
    struct Out {
        std::vector<int32_t> els, nodes;
        std::vector<uint2> recs;
        std::vector<int64_t> cnt, ncnt;
    };
    std::vector<Out> outs(host_threads());
    int used = parallel_chunks(nt, [&](int ci, int64_t tb, int64_t te) {
        Out &o = outs[ci];
        std::vector<int32_t> els, other, nown, idx, sched;
        std::vector<int8_t> vord;
        for (int64_t t = tb; t < te; t++) {
            const int32_t r0 = P.row[t], r1 = P.row[t + 1], nr = r1 - r0;
            els.clear();
            for (int32_t i = r0; i < r1; i++) els.insert(els.end(), n2e.begin() + n2e_ptr[i], n2e.begin() + n2e_ptr[i + 1]);
            std::sort(els.begin(), els.end());
            els.erase(std::unique(els.begin(), els.end()), els.end());
            other.clear();
            for (int32_t e : els)
                for (int a = 0; a < 4; a++) {
                    const int32_t g = m->lnods[4 * (int64_t)e + a];
                    if (g < r0 || g >= r1) other.push_back(g);
                }
            std::sort(other.begin(), other.end());
            other.erase(std::unique(other.begin(), other.end()), other.end());
            for (int32_t i = r0; i < r1; i++) o.nodes.push_back(i);
            o.nodes.insert(o.nodes.end(), other.begin(), other.end());
            o.ncnt.push_back((int64_t)nr + (int64_t)other.size());
            auto local = [&](int32_t g) -> uint32_t {
                if (g >= r0 && g < r1) return (uint32_t)(g - r0);
                return (uint32_t)(nr + (std::lower_bound(other.begin(), other.end(), g) - other.begin()));
            };
            const size_t ne = els.size();
            nown.assign(ne, 0);
            for (size_t j = 0; j < ne; j++)
                for (int a = 0; a < 4; a++) {
                    const int32_t g = m->lnods[4 * (int64_t)els[j] + a];
                    nown[j] += g >= r0 && g < r1;
                }
            idx.resize(ne);
            for (size_t j = 0; j < ne; j++) idx[j] = (int32_t)j;
            std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return nown[x] > nown[y]; });
            // vertex order: owned first, then the others; then the bank-aware order by row
            vord.resize(4 * ne);
            for (size_t j = 0; j < ne; j++) {
                const int32_t *ln = &m->lnods[4 * (int64_t)els[j]];
                int k = 0;
                for (int a = 0; a < 4; a++)
                    if (ln[a] >= r0 && ln[a] < r1) vord[4 * j + k++] = (int8_t)a;
                for (int a = 0; a < 4; a++)
                    if (!(ln[a] >= r0 && ln[a] < r1)) vord[4 * j + k++] = (int8_t)a;
            }
            bank_order(m, els, nown, r0, true, idx, vord, sched);
            idx.swap(sched);
            for (int32_t j : idx) {
                const int32_t *ln = &m->lnods[4 * (int64_t)els[j]];
                uint32_t l[4];
                for (int q = 0; q < 4; q++) l[q] = local(ln[vord[4 * j + q]]);
                o.recs.push_back(make_uint2(l[0] | l[1] << 16, l[2] | l[3] << 16));
                o.els.push_back(els[j]);
            }
            o.cnt.push_back((int64_t)ne);
        }
    });
    P.eptr.assign(1, 0);
    P.nptr.assign(1, 0);
    for (int i = 0; i < used; i++) {
        Out &o = outs[i];
        for (size_t k = 0; k < o.cnt.size(); k++) {
            P.eptr.push_back(P.eptr.back() + o.cnt[k]);
            P.nptr.push_back(P.nptr.back() + o.ncnt[k]);
        }
        P.elems.insert(P.elems.end(), o.els.begin(), o.els.end());
        P.nodes.insert(P.nodes.end(), o.nodes.begin(), o.nodes.end());
        P.recs.insert(P.recs.end(), o.recs.begin(), o.recs.end());
        o = Out();
    }
    if ((int64_t)P.eptr.size() != nt + 1) return fail(NSA_EUNSUPPORTED, "residual plan inconsistent");
    P.ok = true;
    return NSA_OK;
}

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// FP64 geometry of element e in its own vertex order: grad N_0..3 (J^-1 by cofactors, grad N_0 =
// -(grad N_1 + grad N_2 + grad N_3)), V = |det J| / 6, h = |det J|^(1/3), 1/h, 0.
void element_geometry(const nsa_mesh *m, int64_t e, double *g) {
    double X[4][3];
    for (int a = 0; a < 4; a++)
        for (int d = 0; d < 3; d++) X[a][d] = m->coord[3 * (int64_t)m->lnods[4 * e + a] + d];
    double J[3][3];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) J[r][c] = X[c + 1][r] - X[0][r];
    const double cof[3][3] = {{J[1][1] * J[2][2] - J[1][2] * J[2][1], J[1][2] * J[2][0] - J[1][0] * J[2][2],
                               J[1][0] * J[2][1] - J[1][1] * J[2][0]},
                              {J[0][2] * J[2][1] - J[0][1] * J[2][2], J[0][0] * J[2][2] - J[0][2] * J[2][0],
                               J[0][1] * J[2][0] - J[0][0] * J[2][1]},
                              {J[0][1] * J[1][2] - J[0][2] * J[1][1], J[0][2] * J[1][0] - J[0][0] * J[1][2],
                               J[0][0] * J[1][1] - J[0][1] * J[1][0]}};
    const double det = J[0][0] * cof[0][0] + J[0][1] * cof[0][1] + J[0][2] * cof[0][2];
    // grad N_{s+1}[d] = (J^-1)[s][d] = cof[d][s] / det
    for (int s = 0; s < 3; s++)
        for (int d = 0; d < 3; d++) g[3 * (s + 1) + d] = cof[d][s] / det;
    for (int d = 0; d < 3; d++) g[d] = -(g[3 + d] + g[6 + d] + g[9 + d]);
    const double adet = std::fabs(det);
    const double h = std::cbrt(adet);
    g[12] = adet / 6.0;
    g[13] = h;
    g[14] = 1.0 / h;
    g[15] = 0.0;
}

nsa_status q1_plans(nsa_mesh *m);
void q1_layout(nsa_mesh *m);

void plan_layout(nsa_mesh *m) {
    if (m->family == NSA_QUAD4) {
        q1_layout(m);
        return;
    }
    size_t off = 0;
    auto take = [&](nsa::Region &r, size_t bytes) {
        r.off = off;
        r.bytes = bytes;
        off = align_up(off + bytes);
    };
    const size_t ne = (size_t)m->nelem, np = (size_t)m->npoin;
    const bool d = m->keep_direct;
    take(m->r_ln, d ? 4 * ne * sizeof(int32_t) : 0);
    take(m->r_coord, d ? 3 * np * sizeof(double) : 0);
    take(m->r_emap, d ? 16 * ne * sizeof(int32_t) : 0);
    take(m->r_ln_c, d ? 4 * ne * sizeof(int32_t) : 0);
    take(m->r_emap_c, d ? 16 * ne * sizeof(int32_t) : 0);
    const bool t = m->plan[0].ok || m->plan[1].ok || m->gplan.ok || m->rplan.ok;
    // coordinates as 32-byte records: the tiled kernels and the err_out sample read them
    take(m->r_coord4, 4 * np * sizeof(double));
    take(m->r_esamp, (size_t)std::min<int64_t>(m->nelem, NSA_ERR_SAMPLE) * 4 * sizeof(int32_t));
    take(m->r_bptr, t ? (np + 1) * sizeof(int64_t) : 0);
    for (nsa::TilePlan &P : m->plan) {
        take(P.r_row, P.ok ? P.row.size() * sizeof(int32_t) : 0);
        take(P.r_rptr, P.ok ? P.rptr.size() * sizeof(int64_t) : 0);
        take(P.r_nptr, P.ok ? P.nptr.size() * sizeof(int64_t) : 0);
        take(P.r_nodes, P.ok ? P.nodes.size() * sizeof(int32_t) : 0);
        take(P.r_runs, P.ok ? P.runs.size() * sizeof(nsa::RunRec) : 0);
        take(P.r_b0, P.ok ? P.row.size() * sizeof(int64_t) : 0);
        take(P.r_npad, P.ok ? (size_t)P.ntiles() * P.cap_nodes * sizeof(int32_t) : 0);
    }
    nsa::GatherPlan &G = m->gplan;
    take(G.r_row, G.ok ? G.row.size() * sizeof(int32_t) : 0);
    take(G.r_nptr, G.ok ? G.nptr.size() * sizeof(int64_t) : 0);
    take(G.r_nodes, G.ok ? G.nodes.size() * sizeof(int32_t) : 0);
    take(G.r_eptr, G.ok ? G.eptr.size() * sizeof(int64_t) : 0);
    take(G.r_recs, G.ok ? G.recs.size() * sizeof(uint2) : 0);
    take(G.r_pptr, G.ok ? G.pptr.size() * sizeof(int64_t) : 0);
    take(G.r_pairs, G.ok ? G.pairs.size() * sizeof(uint16_t) : 0);
    take(G.r_slots, G.ok ? G.slots.size() * sizeof(uint32_t) : 0);
    nsa::ResPlan &RP = m->rplan;
    take(RP.r_row, RP.ok ? RP.row.size() * sizeof(int32_t) : 0);
    take(RP.r_eptr, RP.ok ? RP.eptr.size() * sizeof(int64_t) : 0);
    take(RP.r_nptr, RP.ok ? RP.nptr.size() * sizeof(int64_t) : 0);
    take(RP.r_nodes, RP.ok ? RP.nodes.size() * sizeof(int32_t) : 0);
    take(RP.r_recs, RP.ok ? RP.recs.size() * sizeof(uint2) : 0);
    const bool geo = RP.ok && m->res_geo_cached;
    take(RP.r_geo, geo ? (size_t)m->nelem * nsa::kGeoDoubles * sizeof(double) : 0);
    take(RP.r_rgel, geo ? RP.recs.size() * sizeof(uint2) : 0);
    m->ws_bytes = std::max<size_t>(off, 256);
}

// Build the requested plans (once) and the device layout. Logically const: called from the read
// accessors of a mesh.
nsa_status ensure_plans(const nsa_mesh *cm) {
    nsa_mesh *m = const_cast<nsa_mesh *>(cm);
    std::lock_guard<std::mutex> g(m->plan_mu);
    if (m->planned) return NSA_OK;
    try {
        if (m->family == NSA_QUAD4) {
            nsa_status st = q1_plans(m);
            if (st) return st;
            m->planned = true;
            return NSA_OK;
        }
        for (int k = 0; k < 2; k++) {
            if (m->want_blocks[k] > 0) {
                nsa_status st = build_tiles(m, m->plan[k], m->want_blocks[k], k == 0 ? m->want_threads : kPlanThreads[k]);
                if (st) return st;
            } else {
                m->plan[k] = nsa::TilePlan();
            }
        }
        if (m->want_gather > 0) {
            nsa_status st = build_gather(m, m->gplan, m->want_gather, kGatherThreads);
            if (st) return st;
        } else {
            m->gplan = nsa::GatherPlan();
        }
        if (m->want_res > 0) {
            nsa_status st = build_rtiles(m, m->rplan, m->want_res);
            if (st) return st;
        } else {
            m->rplan = nsa::ResPlan();
        }
        plan_layout(m);
    } catch (const std::bad_alloc &) {
        return fail(NSA_ENOMEM, "tile planning: host allocation failed");
    }
    m->planned = true;
    return NSA_OK;
}

nsa_status hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) return fail(NSA_EHIP, "%s: %s", what, hipGetErrorString(e));
    return NSA_OK;
}

}  // namespace

// ================================================================================================
// 2-D family: bilinear quadrilaterals
// ================================================================================================
namespace {

// Throughput plan: two-wavefront workgroups on 512-block tiles. The FP64 kernel holds one wave per SIMD,
// so a 256-thread workgroup fills a CU alone and its load, integration and write-out phases never
// overlap; with two waves per workgroup two or more workgroups share a CU (2048^2 quadrilaterals:
// FP64 2.04 -> 1.54 ms; the mixed kernel 1.20 -> 1.22 ms). One-wavefront (deterministic) plan: 256 blocks.
constexpr int32_t kQ1DefaultBlocks[2] = {512, 256};
constexpr int32_t kQ1Threads[2] = {128, 64};

// det J of element e at the four Gauss points (+-1/sqrt 3)^2 of the 2x2 rule: 1 if non-zero, finite
// and of one sign, else 0.
int q1_element_ok(const int32_t *ln, const double *coord) {
    static const double xi[4] = {-1.0, 1.0, 1.0, -1.0}, eta[4] = {-1.0, -1.0, 1.0, 1.0};
    const double g = 1.0 / std::sqrt(3.0);
    int sign = 0;
    for (int gj = 0; gj < 2; gj++)
        for (int gi = 0; gi < 2; gi++) {
            const double x = gi ? g : -g, y = gj ? g : -g;
            double J[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
            for (int a = 0; a < 4; a++) {
                const double d0 = 0.25 * xi[a] * (1.0 + eta[a] * y), d1 = 0.25 * eta[a] * (1.0 + xi[a] * x);
                for (int r = 0; r < 2; r++) {
                    J[r][0] += coord[2 * (int64_t)ln[a] + r] * d0;
                    J[r][1] += coord[2 * (int64_t)ln[a] + r] * d1;
                }
            }
            const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            if (!(det != 0.0) || !std::isfinite(det)) return 0;
            const int sg = det > 0.0 ? 1 : -1;
            if (sign != 0 && sg != sign) return 0;
            sign = sg;
        }
    return 1;
}

// Row tiles of a quadrilateral mesh: contiguous rows whose LDS (q1_lds_bytes) stays within
// tile_blocks * 96 bytes (capped at 160 KB); one record per (element, tile) with an owned vertex.
nsa_status build_q1_tiles(nsa_mesh *m, nsa::Q1Plan &P, int32_t tile_blocks, int32_t threads) {
    P = nsa::Q1Plan();
    P.tile_blocks = tile_blocks;
    P.threads = threads;
    const int64_t np = m->npoin;
    if (np == 0) return NSA_OK;
    const int64_t one_row = nsa::q1_lds_bytes((int32_t)m->max_row_blocks, 1, (int32_t)m->max_row_blocks);
    if (one_row > kMaxTileLds || m->max_row_blocks > 4096) return NSA_OK;
    const int64_t budget = std::max<int64_t>(std::min<int64_t>((int64_t)tile_blocks * 96, kMaxTileLds), one_row);
    std::vector<int32_t> stamp((size_t)np, -1);
    P.row.push_back(0);
    int32_t tid = 0;
    for (int64_t r0 = 0; r0 < np; tid++) {
        int64_t r1 = r0, nodes = 0;
        while (r1 < np) {
            const int64_t add = row_new_nodes(m, stamp, r1, tid);
            const int64_t blocks = m->bptr[r1 + 1] - m->bptr[r0];
            const int64_t need = nsa::q1_lds_bytes((int32_t)blocks, (int32_t)(r1 + 1 - r0), (int32_t)(nodes + add));
            if (r1 > r0 && (need > budget || blocks > 65535 || nodes + add > 65535)) break;
            stamp_row(m, stamp, r1, tid);
            nodes += add;
            r1++;
        }
        P.row.push_back((int32_t)r1);
        P.lds = std::max<int64_t>(P.lds, nsa::q1_lds_bytes((int32_t)(m->bptr[r1] - m->bptr[r0]), (int32_t)(r1 - r0),
                                                          (int32_t)nodes));
        r0 = r1;
    }
    std::vector<int32_t>().swap(stamp);
    const int64_t nt = (int64_t)P.row.size() - 1;
    std::vector<int64_t> n2e_ptr;
    std::vector<int32_t> n2e;
    node_elements(np, m->nelem, m->lnods.data(), n2e_ptr, n2e);
    P.b0.resize((size_t)nt + 1);
    for (int64_t t = 0; t <= nt; t++) P.b0[(size_t)t] = m->bptr[P.row[(size_t)t]];
    P.nptr.assign(1, 0);
    P.eptr.assign(1, 0);
    std::vector<int32_t> els, other;
    for (int64_t t = 0; t < nt; t++) {
        const int32_t r0 = P.row[(size_t)t], r1 = P.row[(size_t)t + 1], nr = r1 - r0;
        els.clear();
        for (int32_t i = r0; i < r1; i++) els.insert(els.end(), n2e.begin() + n2e_ptr[i], n2e.begin() + n2e_ptr[i + 1]);
        std::sort(els.begin(), els.end());
        els.erase(std::unique(els.begin(), els.end()), els.end());
        other.clear();
        for (int32_t e : els)
            for (int a = 0; a < 4; a++) {
                const int32_t g = m->lnods[4 * (int64_t)e + a];
                if (g < r0 || g >= r1) other.push_back(g);
            }
        // a row that no element touches is still owned (it has no blocks to write but an RHS row)
        std::sort(other.begin(), other.end());
        other.erase(std::unique(other.begin(), other.end()), other.end());
        for (int32_t i = r0; i < r1; i++) P.nodes.push_back(i);
        P.nodes.insert(P.nodes.end(), other.begin(), other.end());
        P.nptr.push_back(P.nptr.back() + nr + (int64_t)other.size());
        auto local = [&](int32_t g) -> uint16_t {
            if (g >= r0 && g < r1) return (uint16_t)(g - r0);
            return (uint16_t)(nr + (std::lower_bound(other.begin(), other.end(), g) - other.begin()));
        };
        const int64_t b0 = P.b0[(size_t)t];
        for (int32_t e : els) {
            nsa::Q1Rec r{};
            for (int a = 0; a < 4; a++) {
                const int32_t g = m->lnods[4 * (int64_t)e + a];
                r.loc[a] = local(g);
                if (g >= r0 && g < r1) {
                    r.own |= (uint16_t)(1u << a);
                    for (int b = 0; b < 4; b++) r.slot[4 * a + b] = (uint16_t)(m->emap[16 * (int64_t)e + 4 * a + b] - b0);
                }
            }
            P.recs.push_back(r);
            P.elems.push_back(e);
        }
        P.eptr.push_back((int64_t)P.recs.size());
    }
    P.ok = true;
    return NSA_OK;
}

void q1_layout(nsa_mesh *m) {
    size_t off = 0;
    auto take = [&](nsa::Region &r, size_t bytes) {
        r.off = off;
        r.bytes = bytes;
        off = align_up(off + bytes);
    };
    take(m->r_coord2, 2 * (size_t)m->npoin * sizeof(double));
    for (nsa::Q1Plan &P : m->qplan) {
        take(P.r_row, P.ok ? P.row.size() * sizeof(int32_t) : 0);
        take(P.r_b0, P.ok ? P.b0.size() * sizeof(int64_t) : 0);
        take(P.r_nptr, P.ok ? P.nptr.size() * sizeof(int64_t) : 0);
        take(P.r_nodes, P.ok ? P.nodes.size() * sizeof(int32_t) : 0);
        take(P.r_eptr, P.ok ? P.eptr.size() * sizeof(int64_t) : 0);
        take(P.r_recs, P.ok ? P.recs.size() * sizeof(nsa::Q1Rec) : 0);
    }
    m->ws_bytes = std::max<size_t>(off, 256);
}

nsa_status q1_upload(nsa_mesh *m, char *w, hipStream_t s) {
    try {
        struct Up { const nsa::Region &r; const void *src; };
        std::vector<Up> ups = {{m->r_coord2, m->coord.data()}};
        for (const nsa::Q1Plan &P : m->qplan) {
            if (!P.ok) continue;
            ups.push_back({P.r_row, P.row.data()});
            ups.push_back({P.r_b0, P.b0.data()});
            ups.push_back({P.r_nptr, P.nptr.data()});
            ups.push_back({P.r_nodes, P.nodes.data()});
            ups.push_back({P.r_eptr, P.eptr.data()});
            ups.push_back({P.r_recs, P.recs.data()});
        }
        for (const Up &u : ups) {
            if (!u.r.bytes) continue;
            nsa_status st = hip_check(hipMemcpyAsync(w + u.r.off, u.src, u.r.bytes, hipMemcpyHostToDevice, s), "upload copy");
            if (st) return st;
        }
        nsa_status st = hip_check(hipStreamSynchronize(s), "upload sync");
        if (st) return st;
        int dev = -1;
        st = hip_check(hipGetDevice(&dev), "hipGetDevice");
        if (st) return st;
        m->ws = w;
        m->device = dev;
    } catch (const std::bad_alloc &) {
        return fail(NSA_ENOMEM, "upload: host allocation failed");
    }
    return ok();
}

nsa_status q1_assemble(const nsa_mesh *m, const double *vel, double rho, double mu, double dt, const nsa_options &o,
                       double *values, double *rhs, hipStream_t s) {
    if (o.kernel != NSA_KERNEL_AUTO && o.kernel != NSA_KERNEL_TILED)
        return fail(NSA_EUNSUPPORTED, "quadrilateral meshes take the tiled kernel only");
    if (o.err_out) return fail(NSA_EUNSUPPORTED, "err_out is not available for quadrilateral meshes");
    const nsa::Q1Plan &P = m->qplan[o.scatter];
    if (!P.ok && m->npoin > 0) return fail(NSA_EUNSUPPORTED, "no tile plan for this scatter mode");
    if (o.block_threads != 0 && o.block_threads != P.threads)
        return fail(NSA_EINVAL, "block_threads %d: this plan runs with %d", o.block_threads, P.threads);
    if (!(rho > 0.0) || !std::isfinite(rho) || !(mu >= 0.0) || !std::isfinite(mu) || !(dt > 0.0) || !std::isfinite(dt))
        return fail(NSA_EINVAL, "need rho > 0, mu >= 0, dt > 0 (finite); got %g %g %g", rho, mu, dt);
    if ((m->nelem > 0 && !vel) || (m->nnzb > 0 && !values) || (m->npoin > 0 && !rhs))
        return fail(NSA_EINVAL, "nsa_assemble: null device array");
    if (((uintptr_t)values | (uintptr_t)rhs | (uintptr_t)vel) % 8) return fail(NSA_EINVAL, "arrays must be 8-byte aligned");
    int dev = -1;
    nsa_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st) return st;
    if (dev != m->device) return fail(NSA_EINVAL, "mesh uploaded on device %d, current device is %d", m->device, dev);
    if (m->npoin == 0) return ok();
    nsa::Q1Args a;
    a.ntiles = P.ntiles();
    a.lds_bytes = P.lds;
    a.tile_row = (const int32_t *)(m->ws + P.r_row.off);
    a.tile_b0 = (const int64_t *)(m->ws + P.r_b0.off);
    a.tile_nptr = (const int64_t *)(m->ws + P.r_nptr.off);
    a.tile_nodes = (const int32_t *)(m->ws + P.r_nodes.off);
    a.tile_eptr = (const int64_t *)(m->ws + P.r_eptr.off);
    a.recs = (const uint4 *)(m->ws + P.r_recs.off);
    a.coord = (const double2 *)(m->ws + m->r_coord2.off);
    a.vel = vel;
    a.vel_soa = o.vel_layout == NSA_VEL_SOA ? m->npoin : 0;
    a.rho = rho;
    a.mu = mu;
    a.dt = dt;
    a.accumulate = o.accumulate;
    a.threads = P.threads;
    a.values = values;
    a.rhs = rhs;
    st = hip_check(nsa::launch_q1(o.precision == NSA_MIXED ? nsa::TileKern::Mixed : nsa::TileKern::F64, a, s),
                   "assemble (quadrilaterals)");
    return st ? st : ok();
}

nsa_status q1_plans(nsa_mesh *m) {
    for (int k = 0; k < 2; k++) {
        if (m->want_blocks[k] > 0) {
            nsa_status st = build_q1_tiles(m, m->qplan[k], m->want_blocks[k], kQ1Threads[k]);
            if (st) return st;
        } else {
            m->qplan[k] = nsa::Q1Plan();
        }
    }
    q1_layout(m);
    return NSA_OK;
}

}  // namespace

extern "C" {

const char *nsa_status_string(nsa_status st) {
    switch (st) {
        case NSA_OK: return "ok";
        case NSA_EINVAL: return "invalid argument";
        case NSA_ERANGE: return "connectivity entry out of range";
        case NSA_EDEGENERATE: return "degenerate element";
        case NSA_ENOMEM: return "out of memory or buffer too small";
        case NSA_EHIP: return "HIP runtime error";
        case NSA_EUNSUPPORTED: return "unsupported";
        case NSA_ESTATE: return "call out of order";
        default: return "unknown status";
    }
}

const char *nsa_last_error(void) { return g_last_error; }

int32_t nsa_version(void) { return 310; }

nsa_status nsa_pattern_count(int64_t npoin, int64_t nelem, const int32_t *lnods, int64_t *bptr,
                             int64_t *nnzb) {
    if (npoin < 0 || nelem < 0 || !bptr || !nnzb || (nelem > 0 && !lnods))
        return fail(NSA_EINVAL, "nsa_pattern_count: bad arguments");
    if (nelem > INT32_MAX || npoin > INT32_MAX)
        return fail(NSA_EUNSUPPORTED, "more than 2^31-1 nodes or elements");
    try {
        nsa_status st = check_range(npoin, nelem, lnods);
        if (st) return st;
        std::vector<int64_t> ptr;
        std::vector<int32_t> list;
        node_elements(npoin, nelem, lnods, ptr, list);
        std::vector<int64_t> bp;
        pattern_rows(npoin, lnods, ptr, list, bp, nullptr);
        std::copy(bp.begin(), bp.end(), bptr);
        *nnzb = bp[npoin];
    } catch (const std::bad_alloc &) {
        return fail(NSA_ENOMEM, "nsa_pattern_count: host allocation failed");
    }
    return ok();
}

nsa_status nsa_pattern_fill(int64_t npoin, int64_t nelem, const int32_t *lnods, const int64_t *bptr,
                            int32_t *bcol, int32_t *emap) {
    if (npoin < 0 || nelem < 0 || !bptr || !bcol || (nelem > 0 && !lnods))
        return fail(NSA_EINVAL, "nsa_pattern_fill: bad arguments");
    try {
        nsa_status st = check_range(npoin, nelem, lnods);
        if (st) return st;
        std::vector<int64_t> ptr;
        std::vector<int32_t> list;
        node_elements(npoin, nelem, lnods, ptr, list);
        std::vector<int64_t> bp(bptr, bptr + npoin + 1);
        std::vector<int32_t> bc(bp[npoin]);
        pattern_rows(npoin, lnods, ptr, list, bp, &bc);
        std::copy(bc.begin(), bc.end(), bcol);
        if (emap) fill_emap(nelem, lnods, bptr, bcol, emap);
    } catch (const std::bad_alloc &) {
        return fail(NSA_ENOMEM, "nsa_pattern_fill: host allocation failed");
    }
    return ok();
}

nsa_status nsa_mesh_create(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord,
                           nsa_mesh **out) {
    if (!out || npoin < 0 || nelem < 0 || (nelem > 0 && !lnods) || (npoin > 0 && !coord))
        return fail(NSA_EINVAL, "nsa_mesh_create: bad arguments");
    if (nelem > INT32_MAX || npoin > INT32_MAX)
        return fail(NSA_EUNSUPPORTED, "more than 2^31-1 nodes or elements");
    *out = nullptr;
    nsa_mesh *m = nullptr;
    try {
        nsa_status st = check_range(npoin, nelem, lnods);
        if (st) return st;
        std::atomic<int64_t> bad{-1};
        parallel_for(nelem, [&](int64_t b, int64_t e) {
            for (int64_t i = b; i < e; i++) {
                double det = elem_det(lnods + 4 * i, coord);
                if (!(det != 0.0) || !std::isfinite(det)) {
                    int64_t cur = bad.load();
                    while ((cur < 0 || i < cur) && !bad.compare_exchange_weak(cur, i)) {
                    }
                }
            }
        });
        if (bad.load() >= 0)
            return fail(NSA_EDEGENERATE, "element %lld has a zero or non-finite Jacobian determinant",
                        (long long)bad.load());
        m = new nsa_mesh;
        m->npoin = npoin;
        m->nelem = nelem;
        m->lnods.assign(lnods, lnods + 4 * nelem);
        m->coord.assign(coord, coord + 3 * npoin);
        std::vector<int64_t> ptr;
        std::vector<int32_t> list;
        node_elements(npoin, nelem, lnods, ptr, list);
        pattern_rows(npoin, lnods, ptr, list, m->bptr, nullptr);
        m->nnzb = m->bptr[npoin];
        if (m->nnzb > INT32_MAX) {
            delete m;
            return fail(NSA_EUNSUPPORTED, "more than 2^31-1 blocks");
        }
        m->bcol.resize(m->nnzb);
        pattern_rows(npoin, lnods, ptr, list, m->bptr, &m->bcol);
        for (int64_t i = 0; i < npoin; i++)
            m->max_row_blocks = std::max(m->max_row_blocks, m->bptr[i + 1] - m->bptr[i]);
        m->emap.resize(16 * (size_t)nelem);
        fill_emap(nelem, lnods, m->bptr.data(), m->bcol.data(), m->emap.data());
        st = colour_elements(m);
        m->want_blocks[0] = kDefaultTileBlocks[0];
        m->want_blocks[1] = kDefaultTileBlocks[1];
        m->want_gather = 0;  // the gather plan is opt-in (nsa_mesh_set_tiling with NSA_GATHER_PLAN)
        if (st) {
            delete m;
            return st;
        }
    } catch (const std::bad_alloc &) {
        delete m;
        return fail(NSA_ENOMEM, "nsa_mesh_create: host allocation failed");
    }
    *out = m;
    return ok();
}

nsa_status nsa_mesh_create_q1(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord,
                              nsa_mesh **out) {
    if (!out || npoin < 0 || nelem < 0 || (nelem > 0 && !lnods) || (npoin > 0 && !coord))
        return fail(NSA_EINVAL, "nsa_mesh_create_q1: bad arguments");
    if (nelem > INT32_MAX || npoin > INT32_MAX) return fail(NSA_EUNSUPPORTED, "more than 2^31-1 nodes or elements");
    *out = nullptr;
    nsa_mesh *m = nullptr;
    try {
        nsa_status st = check_range(npoin, nelem, lnods);
        if (st) return st;
        std::atomic<int64_t> bad{-1};
        parallel_for(nelem, [&](int64_t b, int64_t e) {
            for (int64_t i = b; i < e; i++)
                if (!q1_element_ok(lnods + 4 * i, coord)) {
                    int64_t cur = bad.load();
                    while ((cur < 0 || i < cur) && !bad.compare_exchange_weak(cur, i)) {
                    }
                }
        });
        if (bad.load() >= 0)
            return fail(NSA_EDEGENERATE, "quadrilateral %lld: det J zero, not finite or of changing sign at its Gauss points",
                        (long long)bad.load());
        m = new nsa_mesh;
        m->family = NSA_QUAD4;
        m->npoin = npoin;
        m->nelem = nelem;
        m->keep_direct = false;
        m->lnods.assign(lnods, lnods + 4 * nelem);
        m->coord.assign(coord, coord + 2 * npoin);
        std::vector<int64_t> ptr;
        std::vector<int32_t> list;
        node_elements(npoin, nelem, lnods, ptr, list);
        pattern_rows(npoin, lnods, ptr, list, m->bptr, nullptr);
        m->nnzb = m->bptr[npoin];
        if (m->nnzb > INT32_MAX) {
            delete m;
            return fail(NSA_EUNSUPPORTED, "more than 2^31-1 blocks");
        }
        m->bcol.resize(m->nnzb);
        pattern_rows(npoin, lnods, ptr, list, m->bptr, &m->bcol);
        for (int64_t i = 0; i < npoin; i++)
            m->max_row_blocks = std::max(m->max_row_blocks, m->bptr[i + 1] - m->bptr[i]);
        m->emap.resize(16 * (size_t)nelem);
        fill_emap(nelem, lnods, m->bptr.data(), m->bcol.data(), m->emap.data());
        m->want_blocks[0] = kQ1DefaultBlocks[0];
        m->want_blocks[1] = kQ1DefaultBlocks[1];
    } catch (const std::bad_alloc &) {
        delete m;
        return fail(NSA_ENOMEM, "nsa_mesh_create_q1: host allocation failed");
    }
    *out = m;
    return ok();
}

nsa_status nsa_mesh_get_q1_tiles(const nsa_mesh *m, int32_t scatter, int32_t *tile_row, int64_t *tile_eptr,
                                 int32_t *elems, void *recs, int64_t *tile_nptr, int32_t *tile_nodes) {
    if (!m) return fail(NSA_EINVAL, "nsa_mesh_get_q1_tiles: null mesh");
    if (m->family != NSA_QUAD4) return fail(NSA_EUNSUPPORTED, "nsa_mesh_get_q1_tiles: not a quadrilateral mesh");
    if (scatter != NSA_ATOMIC && scatter != NSA_COLOUR) return fail(NSA_EINVAL, "unknown scatter mode %d", scatter);
    if (m->host_released) return fail(NSA_ESTATE, "host copy released");
    nsa_status st = ensure_plans(m);
    if (st) return st;
    const nsa::Q1Plan &P = m->qplan[scatter];
    if (!P.ok) return fail(NSA_EUNSUPPORTED, "no tile plan for scatter mode %d", scatter);
    if (tile_row) std::copy(P.row.begin(), P.row.end(), tile_row);
    if (tile_eptr) std::copy(P.eptr.begin(), P.eptr.end(), tile_eptr);
    if (elems) std::copy(P.elems.begin(), P.elems.end(), elems);
    if (recs) std::memcpy(recs, P.recs.data(), P.recs.size() * sizeof(nsa::Q1Rec));
    if (tile_nptr) std::copy(P.nptr.begin(), P.nptr.end(), tile_nptr);
    if (tile_nodes) std::copy(P.nodes.begin(), P.nodes.end(), tile_nodes);
    return ok();
}

nsa_status nsa_mesh_set_tiling(nsa_mesh *m, int32_t scatter, int32_t tile_blocks) {
    if (!m) return fail(NSA_EINVAL, "nsa_mesh_set_tiling: null mesh");
    if (m->family == NSA_QUAD4 && (scatter == NSA_GATHER_PLAN || scatter == NSA_RESIDUAL_PLAN))
        return fail(NSA_EUNSUPPORTED, "quadrilateral meshes have row-tile plans for NSA_ATOMIC and NSA_COLOUR only");
    if (scatter != NSA_ATOMIC && scatter != NSA_COLOUR && scatter != NSA_GATHER_PLAN && scatter != NSA_RESIDUAL_PLAN)
        return fail(NSA_EINVAL, "unknown plan %d", scatter);
    if (scatter == NSA_RESIDUAL_PLAN) {
        if (tile_blocks != 0 && (tile_blocks < 1 || tile_blocks > kMaxResRows))
            return fail(NSA_EINVAL, "rows per residual tile %d outside [1, %d] (or 0)", tile_blocks, kMaxResRows);
    } else {
        const int32_t cap = scatter == NSA_GATHER_PLAN ? kMaxGatherBlocks : kMaxTileBlocks;
        if (tile_blocks != 0 && (tile_blocks < 64 || tile_blocks > cap))
            return fail(NSA_EINVAL, "tile_blocks %d outside [64, %d] (or 0)", tile_blocks, cap);
    }
    if (m->ws || m->host_released) return fail(NSA_ESTATE, "nsa_mesh_set_tiling after upload");
    std::lock_guard<std::mutex> g(m->plan_mu);
    if (scatter == NSA_RESIDUAL_PLAN) {
        if (m->want_res != tile_blocks || !m->planned) {
            m->want_res = tile_blocks;
            m->planned = false;
        }
        return ok();
    }
    if (scatter == NSA_GATHER_PLAN) {
        if (m->want_gather != tile_blocks || !m->planned) {
            m->want_gather = tile_blocks;
            m->planned = false;
        }
        return ok();
    }
    if (m->want_blocks[scatter] != tile_blocks || !m->planned) {
        m->want_blocks[scatter] = tile_blocks;
        m->planned = false;
    }
    return ok();
}

nsa_status nsa_mesh_set_tile_threads(nsa_mesh *m, int32_t threads) {
    if (!m || (threads != 64 && threads != 128 && threads != 192 && threads != 256))
        return fail(NSA_EINVAL, "nsa_mesh_set_tile_threads: threads must be 64, 128, 192 or 256");
    if (m->family == NSA_QUAD4) return fail(NSA_EUNSUPPORTED, "%s is not available for quadrilateral meshes", __func__);
    if (m->ws || m->host_released) return fail(NSA_ESTATE, "nsa_mesh_set_tile_threads after upload");
    std::lock_guard<std::mutex> g(m->plan_mu);
    if (m->want_threads != threads) {
        m->want_threads = threads;
        m->planned = false;
    }
    return ok();
}

nsa_status nsa_mesh_keep_direct(nsa_mesh *m, int32_t keep) {
    if (!m || (keep != 0 && keep != 1)) return fail(NSA_EINVAL, "nsa_mesh_keep_direct: bad arguments");
    if (m->family == NSA_QUAD4) return fail(NSA_EUNSUPPORTED, "%s is not available for quadrilateral meshes", __func__);
    if (m->ws || m->host_released) return fail(NSA_ESTATE, "nsa_mesh_keep_direct after upload");
    std::lock_guard<std::mutex> g(m->plan_mu);
    if (m->keep_direct != (keep == 1)) {
        m->keep_direct = keep == 1;
        if (m->planned) plan_layout(m);  // tile plans stay; only the workspace layout changes
    }
    return ok();
}

nsa_status nsa_mesh_set_residual_geometry(nsa_mesh *m, int32_t cached) {
    if (!m || (cached != 0 && cached != 1)) return fail(NSA_EINVAL, "nsa_mesh_set_residual_geometry: bad arguments");
    if (m->family == NSA_QUAD4) return fail(NSA_EUNSUPPORTED, "%s is not available for quadrilateral meshes", __func__);
    if (m->ws || m->host_released) return fail(NSA_ESTATE, "nsa_mesh_set_residual_geometry after upload");
    std::lock_guard<std::mutex> g(m->plan_mu);
    if (m->res_geo_cached != (cached == 1)) {
        m->res_geo_cached = cached == 1;
        if (m->planned) plan_layout(m);
    }
    return ok();
}

nsa_status nsa_mesh_destroy(nsa_mesh *m) {
    delete m;
    return ok();
}

nsa_status nsa_mesh_get_info(const nsa_mesh *m, nsa_mesh_info *info) {
    if (!m || !info) return fail(NSA_EINVAL, "nsa_mesh_get_info: null argument");
    if (!m->host_released) {
        nsa_status st = ensure_plans(m);
        if (st) return st;
    }
    info->family = m->family;
    info->pad0 = 0;
    info->npoin = m->npoin;
    info->nelem = m->nelem;
    info->nnzb = m->nnzb;
    info->ncolours = m->ncolours;
    info->uploaded = m->ws != nullptr;
    info->ws_bytes = m->ws_bytes;
    info->max_row_blocks = m->max_row_blocks;
    for (int k = 0; k < 2; k++) {
        const nsa::TilePlan &P = m->plan[k];
        info->ntiles[k] = P.ntiles();
        info->tile_runs[k] = P.nruns();
        info->tile_blocks[k] = P.tile_blocks;
        info->tile_threads[k] = P.threads;
        info->tile_max_runs[k] = P.cap_runs;
        info->tile_lds_bytes[k] = P.ok ? (int32_t)P.lds : 0;
    }
    if (m->family == NSA_QUAD4)
        for (int k = 0; k < 2; k++) {
            const nsa::Q1Plan &Q = m->qplan[k];
            info->ntiles[k] = Q.ntiles();
            info->tile_runs[k] = Q.ok ? (int64_t)Q.recs.size() : 0;  // (element, tile) records
            info->tile_blocks[k] = Q.tile_blocks;
            info->tile_threads[k] = Q.threads;
            info->tile_max_runs[k] = 0;
            info->tile_lds_bytes[k] = Q.ok ? (int32_t)Q.lds : 0;
        }
    const nsa::GatherPlan &G = m->gplan;
    info->gather_ntiles = G.ntiles();
    info->gather_records = G.ok ? G.eptr.back() : 0;
    info->gather_pairs = G.ok ? G.pptr.back() : 0;
    info->gather_tile_blocks = G.tile_blocks;
    info->gather_threads = G.threads;
    info->gather_lds_bytes[0] = G.ok ? (int32_t)G.lds[0] : 0;
    info->gather_lds_bytes[1] = G.ok ? (int32_t)G.lds[1] : 0;
    const nsa::ResPlan &RP = m->rplan;
    info->residual_ntiles = RP.ntiles();
    info->residual_records = RP.ok ? RP.eptr.back() : 0;
    info->residual_tile_rows = RP.tile_rows;
    info->residual_lds_bytes = RP.ok ? (int32_t)RP.lds : 0;
    return ok();
}

nsa_status nsa_mesh_get_pattern(const nsa_mesh *m, int64_t *bptr, int32_t *bcol, int32_t *emap) {
    if (!m) return fail(NSA_EINVAL, "nsa_mesh_get_pattern: null mesh");
    if (m->host_released) return fail(NSA_ESTATE, "host copy released");
    if (bptr) std::copy(m->bptr.begin(), m->bptr.end(), bptr);
    if (bcol) std::copy(m->bcol.begin(), m->bcol.end(), bcol);
    if (emap) std::copy(m->emap.begin(), m->emap.end(), emap);
    return ok();
}

nsa_status nsa_pattern_scalar_csr(const nsa_mesh *m, int64_t *row_ptr, int32_t *col) {
    if (!m) return fail(NSA_EINVAL, "nsa_pattern_scalar_csr: null mesh");
    if (m->family == NSA_QUAD4) return fail(NSA_EUNSUPPORTED, "%s is not available for quadrilateral meshes", __func__);
    if (m->host_released) return fail(NSA_ESTATE, "host copy released");
    if (4 * m->npoin > INT32_MAX) return fail(NSA_EUNSUPPORTED, "scalar columns exceed int32");
    if (row_ptr) {
        for (int64_t i = 0; i < m->npoin; i++) {
            const int64_t deg = m->bptr[i + 1] - m->bptr[i];
            for (int c = 0; c < 4; c++) row_ptr[4 * i + c] = 16 * m->bptr[i] + 4 * c * deg;
        }
        row_ptr[4 * m->npoin] = 16 * m->nnzb;
    }
    if (col) {
        parallel_for(m->npoin, [&](int64_t b, int64_t e) {
            for (int64_t i = b; i < e; i++) {
                const int64_t k0 = m->bptr[i], deg = m->bptr[i + 1] - k0;
                for (int c = 0; c < 4; c++) {
                    int32_t *out = col + 16 * k0 + 4 * c * deg;
                    for (int64_t k = 0; k < deg; k++)
                        for (int cp = 0; cp < 4; cp++) out[4 * k + cp] = 4 * m->bcol[k0 + k] + cp;
                }
            }
        }, 1024);
    }
    return ok();
}

nsa_status nsa_mesh_get_colouring(const nsa_mesh *m, int32_t *colour_ptr, int32_t *colour_elems) {
    if (!m) return fail(NSA_EINVAL, "nsa_mesh_get_colouring: null mesh");
    if (m->family == NSA_QUAD4) return fail(NSA_EUNSUPPORTED, "%s is not available for quadrilateral meshes", __func__);
    if (m->host_released) return fail(NSA_ESTATE, "host copy released");
    if (colour_ptr) std::copy(m->colour_ptr.begin(), m->colour_ptr.end(), colour_ptr);
    if (colour_elems) std::copy(m->colour_elems.begin(), m->colour_elems.end(), colour_elems);
    return ok();
}

nsa_status nsa_mesh_get_tiles(const nsa_mesh *m, int32_t scatter, int32_t *tile_row, int64_t *tile_rptr,
                              int32_t *run_elems, int64_t *tile_nptr, int32_t *tile_nodes, uint8_t *runs) {
    if (!m) return fail(NSA_EINVAL, "nsa_mesh_get_tiles: null mesh");
    if (m->family == NSA_QUAD4) return fail(NSA_EUNSUPPORTED, "%s is not available for quadrilateral meshes", __func__);
    if (scatter != NSA_ATOMIC && scatter != NSA_COLOUR) return fail(NSA_EINVAL, "unknown scatter mode %d", scatter);
    if (m->host_released) return fail(NSA_ESTATE, "host copy released");
    nsa_status st = ensure_plans(m);
    if (st) return st;
    const nsa::TilePlan &P = m->plan[scatter];
    if (!P.ok) return fail(NSA_EUNSUPPORTED, "no tile plan for this mesh");
    if (tile_row) std::copy(P.row.begin(), P.row.end(), tile_row);
    if (tile_rptr) std::copy(P.rptr.begin(), P.rptr.end(), tile_rptr);
    if (run_elems) std::copy(P.relems.begin(), P.relems.end(), run_elems);
    if (tile_nptr) std::copy(P.nptr.begin(), P.nptr.end(), tile_nptr);
    if (tile_nodes) std::copy(P.nodes.begin(), P.nodes.end(), tile_nodes);
    if (runs) std::memcpy(runs, P.runs.data(), P.runs.size() * sizeof(nsa::RunRec));
    return ok();
}

nsa_status nsa_mesh_get_gather(const nsa_mesh *m, int32_t *tile_row, int64_t *tile_nptr, int32_t *tile_nodes,
                               int64_t *tile_eptr, int32_t *elems, uint16_t *local_nodes, int64_t *tile_pptr,
                               uint16_t *pairs, uint32_t *slots) {
    if (!m) return fail(NSA_EINVAL, "nsa_mesh_get_gather: null mesh");
    if (m->family == NSA_QUAD4) return fail(NSA_EUNSUPPORTED, "%s is not available for quadrilateral meshes", __func__);
    if (m->host_released) return fail(NSA_ESTATE, "host copy released");
    nsa_status st = ensure_plans(m);
    if (st) return st;
    const nsa::GatherPlan &G = m->gplan;
    if (!G.ok) return fail(NSA_EUNSUPPORTED, "no gather plan for this mesh");
    if (tile_row) std::copy(G.row.begin(), G.row.end(), tile_row);
    if (tile_nptr) std::copy(G.nptr.begin(), G.nptr.end(), tile_nptr);
    if (tile_nodes) std::copy(G.nodes.begin(), G.nodes.end(), tile_nodes);
    if (tile_eptr) std::copy(G.eptr.begin(), G.eptr.end(), tile_eptr);
    if (elems) std::copy(G.elems.begin(), G.elems.end(), elems);
    if (local_nodes) std::memcpy(local_nodes, G.recs.data(), G.recs.size() * sizeof(uint2));
    if (tile_pptr) std::copy(G.pptr.begin(), G.pptr.end(), tile_pptr);
    if (pairs) std::copy(G.pairs.begin(), G.pairs.end(), pairs);
    if (slots) std::copy(G.slots.begin(), G.slots.end(), slots);
    return ok();
}

nsa_status nsa_mesh_get_residual_tiles(const nsa_mesh *m, int32_t *tile_row, int64_t *tile_eptr, int32_t *elems,
                                       uint16_t *local_nodes, int64_t *tile_nptr, int32_t *tile_nodes) {
    if (!m) return fail(NSA_EINVAL, "nsa_mesh_get_residual_tiles: null mesh");
    if (m->family == NSA_QUAD4) return fail(NSA_EUNSUPPORTED, "%s is not available for quadrilateral meshes", __func__);
    if (m->host_released) return fail(NSA_ESTATE, "host copy released");
    nsa_status st = ensure_plans(m);
    if (st) return st;
    const nsa::ResPlan &RP = m->rplan;
    if (!RP.ok) return fail(NSA_EUNSUPPORTED, "no residual plan for this mesh");
    if (tile_row) std::copy(RP.row.begin(), RP.row.end(), tile_row);
    if (tile_eptr) std::copy(RP.eptr.begin(), RP.eptr.end(), tile_eptr);
    if (elems) std::copy(RP.elems.begin(), RP.elems.end(), elems);
    if (local_nodes) std::memcpy(local_nodes, RP.recs.data(), RP.recs.size() * sizeof(uint2));
    if (tile_nptr) std::copy(RP.nptr.begin(), RP.nptr.end(), tile_nptr);
    if (tile_nodes) std::copy(RP.nodes.begin(), RP.nodes.end(), tile_nodes);
    return ok();
}

nsa_status nsa_mesh_upload(nsa_mesh *m, void *ws, size_t ws_bytes, void *stream) {
    if (!m || !ws) return fail(NSA_EINVAL, "nsa_mesh_upload: null argument");
    if (m->host_released) return fail(NSA_ESTATE, "host copy released");
    {
        nsa_status st0 = ensure_plans(m);
        if (st0) return st0;
    }
    if (ws_bytes < m->ws_bytes)
        return fail(NSA_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, m->ws_bytes);
    if (((uintptr_t)ws) % 256) return fail(NSA_EINVAL, "workspace not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    if (m->family == NSA_QUAD4) return q1_upload(m, (char *)ws, s);
    const int64_t ne = m->nelem, np = m->npoin;
    try {
        const bool d = m->keep_direct;
        std::vector<int32_t> ln(d ? 4 * ne : 0), em(d ? 16 * ne : 0), lnc(d ? 4 * ne : 0), emc(d ? 16 * ne : 0);
        std::vector<double> co(d ? 3 * np : 0);
        if (d) parallel_for(ne, [&](int64_t b, int64_t e) {
            for (int64_t i = b; i < e; i++) {
                for (int a = 0; a < 4; a++) ln[a * ne + i] = m->lnods[4 * i + a];
                for (int k = 0; k < 16; k++) em[k * ne + i] = m->emap[16 * i + k];
                int64_t src = m->colour_elems[i];
                for (int a = 0; a < 4; a++) lnc[a * ne + i] = m->lnods[4 * src + a];
                for (int k = 0; k < 16; k++) emc[k * ne + i] = m->emap[16 * src + k];
            }
        });
        if (d)
            for (int64_t i = 0; i < np; i++)
                for (int c = 0; c < 3; c++) co[c * np + i] = m->coord[3 * i + c];
        std::vector<double> co4(4 * (size_t)np, 0.0);
        for (int64_t i = 0; i < np; i++)
            for (int d = 0; d < 3; d++) co4[4 * i + d] = m->coord[3 * i + d];
        // err_out sample: element floor(i nelem / ns) for i < ns, its four node ids
        const int64_t ns = std::min<int64_t>(ne, NSA_ERR_SAMPLE);
        std::vector<int32_t> esamp(4 * (size_t)ns);
        for (int64_t i = 0; i < ns; i++) {
            const int64_t e = i * ne / ns;
            for (int a = 0; a < 4; a++) esamp[4 * i + a] = m->lnods[4 * e + a];
        }
        // per plan: block offset of each tile and its node ids at a fixed stride (padding repeats
        // the tile's first node, so every padded gather stays inside the mesh)
        std::vector<int64_t> b0v[2];
        std::vector<int32_t> npad[2];
        for (int k = 0; k < 2; k++) {
            const nsa::TilePlan &P = m->plan[k];
            if (!P.ok) continue;
            b0v[k].resize(P.row.size());
            for (size_t t = 0; t < P.row.size(); t++) b0v[k][t] = m->bptr[P.row[t]];
            const int64_t nt = P.ntiles(), cap = P.cap_nodes;
            npad[k].resize((size_t)(nt * cap));
            for (int64_t t = 0; t < nt; t++) {
                const int64_t a = P.nptr[t], n = P.nptr[t + 1] - a;
                for (int64_t i = 0; i < cap; i++) npad[k][t * cap + i] = P.nodes[a + (i < n ? i : 0)];
            }
        }
        // precomputed residual geometry: per element (own vertex order) the FP64 gradients, volume,
        // length and inverse length; per record the element and the element vertex of each local vertex
        std::vector<double> geo;
        std::vector<uint2> rgel;
        const nsa::ResPlan &RG = m->rplan;
        if (RG.ok && m->res_geo_cached) {
            geo.assign((size_t)ne * nsa::kGeoDoubles, 0.0);
            parallel_for(ne, [&](int64_t b, int64_t e) {
                for (int64_t i = b; i < e; i++) element_geometry(m, i, &geo[(size_t)i * nsa::kGeoDoubles]);
            });
            rgel.resize(RG.recs.size());
            const int64_t nt = RG.ntiles();
            parallel_for(nt, [&](int64_t tb, int64_t te) {
                for (int64_t t = tb; t < te; t++)
                    for (int64_t p = RG.eptr[t]; p < RG.eptr[t + 1]; p++) {
                        const int32_t el = RG.elems[p];
                        const uint2 r = RG.recs[p];
                        const uint32_t loc[4] = {r.x & 0xffffu, r.x >> 16, r.y & 0xffffu, r.y >> 16};
                        uint32_t perm = 0;
                        for (int a = 0; a < 4; a++) {
                            const int32_t g = RG.nodes[RG.nptr[t] + loc[a]];
                            int v = 0;
                            while (v < 4 && m->lnods[4 * (int64_t)el + v] != g) v++;
                            perm |= (uint32_t)(v & 3) << (2 * a);
                        }
                        rgel[p] = make_uint2((uint32_t)el, perm);
                    }
            });
        }
        char *w = (char *)ws;
        nsa_status st;
        struct Up { const nsa::Region &r; const void *src; };
        const nsa::TilePlan &P0 = m->plan[0], &P1 = m->plan[1];
        const nsa::GatherPlan &G = m->gplan;
        const nsa::ResPlan &RP = m->rplan;
        const Up ups[] = {{m->r_ln, ln.data()}, {m->r_coord, co.data()}, {m->r_emap, em.data()},
                          {m->r_ln_c, lnc.data()}, {m->r_emap_c, emc.data()},
                          {m->r_coord4, co4.data()}, {m->r_esamp, esamp.data()}, {m->r_bptr, m->bptr.data()},
                          {P0.r_row, P0.row.data()}, {P0.r_rptr, P0.rptr.data()}, {P0.r_nptr, P0.nptr.data()},
                          {P0.r_nodes, P0.nodes.data()}, {P0.r_runs, P0.runs.data()},
                          {P0.r_b0, b0v[0].data()}, {P0.r_npad, npad[0].data()},
                          {P1.r_row, P1.row.data()}, {P1.r_rptr, P1.rptr.data()}, {P1.r_nptr, P1.nptr.data()},
                          {P1.r_nodes, P1.nodes.data()}, {P1.r_runs, P1.runs.data()},
                          {P1.r_b0, b0v[1].data()}, {P1.r_npad, npad[1].data()},
                          {G.r_row, G.row.data()}, {G.r_nptr, G.nptr.data()}, {G.r_nodes, G.nodes.data()},
                          {G.r_eptr, G.eptr.data()}, {G.r_recs, G.recs.data()}, {G.r_pptr, G.pptr.data()},
                          {G.r_pairs, G.pairs.data()}, {G.r_slots, G.slots.data()},
                          {RP.r_row, RP.row.data()}, {RP.r_eptr, RP.eptr.data()}, {RP.r_nptr, RP.nptr.data()},
                          {RP.r_nodes, RP.nodes.data()}, {RP.r_recs, RP.recs.data()},
                          {RP.r_geo, geo.data()}, {RP.r_rgel, rgel.data()}};
        for (const Up &u : ups) {
            if (!u.r.bytes) continue;
            st = hip_check(hipMemcpyAsync(w + u.r.off, u.src, u.r.bytes, hipMemcpyHostToDevice, s),
                           "upload copy");
            if (st) return st;
        }
        st = hip_check(hipStreamSynchronize(s), "upload sync");
        if (st) return st;
        int dev = -1;
        st = hip_check(hipGetDevice(&dev), "hipGetDevice");
        if (st) return st;
        m->ws = w;
        m->device = dev;
    } catch (const std::bad_alloc &) {
        return fail(NSA_ENOMEM, "nsa_mesh_upload: host allocation failed");
    }
    return ok();
}

nsa_status nsa_mesh_release_host(nsa_mesh *m) {
    if (!m) return fail(NSA_EINVAL, "nsa_mesh_release_host: null mesh");
    if (!m->ws) return fail(NSA_ESTATE, "release before upload");
    std::vector<int32_t>().swap(m->lnods);
    std::vector<double>().swap(m->coord);
    std::vector<int32_t>().swap(m->bcol);
    std::vector<int32_t>().swap(m->emap);
    std::vector<int32_t>().swap(m->colour_elems);
    {
        nsa::ResPlan &RP = m->rplan;
        std::vector<int32_t>().swap(RP.elems);
        std::vector<int32_t>().swap(RP.nodes);
        std::vector<uint2>().swap(RP.recs);
    }
    {
        nsa::GatherPlan &G = m->gplan;
        std::vector<int32_t>().swap(G.elems);
        std::vector<int32_t>().swap(G.nodes);
        std::vector<uint2>().swap(G.recs);
        std::vector<uint16_t>().swap(G.pairs);
        std::vector<uint32_t>().swap(G.slots);
    }
    for (nsa::TilePlan &P : m->plan) {
        std::vector<int32_t>().swap(P.relems);
        std::vector<int32_t>().swap(P.nodes);
        std::vector<nsa::RunRec>().swap(P.runs);
    }
    m->host_released = true;
    return ok();
}

namespace {
nsa_status assemble_impl(const nsa_mesh *m, const double *vel, double rho, double mu, double dt,
                         const nsa_options *opt, double *values, double *rhs, void *stream) {
    if (!m) return fail(NSA_EINVAL, "nsa_assemble: null mesh");
    if (!m->ws) return fail(NSA_ESTATE, "nsa_assemble: mesh not uploaded");
    nsa_options o{};
    if (opt) o = *opt;
    if (o.precision != NSA_FP64 && o.precision != NSA_MIXED)
        return fail(NSA_EINVAL, "unknown precision %d", o.precision);
    if (o.scatter != NSA_ATOMIC && o.scatter != NSA_COLOUR)
        return fail(NSA_EINVAL, "unknown scatter mode %d", o.scatter);
    if (o.accumulate != 0 && o.accumulate != 1) return fail(NSA_EINVAL, "accumulate must be 0 or 1");
    if (o.vel_layout != NSA_VEL_AOS && o.vel_layout != NSA_VEL_SOA)
        return fail(NSA_EINVAL, "unknown velocity layout %d", o.vel_layout);
    if (o.kernel != NSA_KERNEL_AUTO && o.kernel != NSA_KERNEL_TILED && o.kernel != NSA_KERNEL_DIRECT &&
        o.kernel != NSA_KERNEL_GATHER)
        return fail(NSA_EINVAL, "unknown kernel %d", o.kernel);
    if ((uintptr_t)o.err_out % 8) return fail(NSA_EINVAL, "err_out must be 8-byte aligned");
    if (m->family == NSA_QUAD4) return q1_assemble(m, vel, rho, mu, dt, o, values, rhs, (hipStream_t)stream);
    const int64_t vsoa = o.vel_layout == NSA_VEL_SOA ? m->npoin : 0;
    const nsa::TilePlan &P = m->plan[o.scatter];
    const nsa::GatherPlan &G = m->gplan;
    if (o.kernel == NSA_KERNEL_TILED && !P.ok)
        return fail(NSA_EUNSUPPORTED, "this mesh cannot use the tiled kernel (row degree > 256 or no plan)");
    if (o.kernel == NSA_KERNEL_GATHER && !G.ok)
        return fail(NSA_EUNSUPPORTED, "this mesh has no gather plan");
    int threads = o.block_threads ? o.block_threads : 256;
    if (o.kernel == NSA_KERNEL_GATHER) {
        if (threads != 256 && threads != 512)
            return fail(NSA_EINVAL, "block_threads %d: the gather kernel takes 256 or 512", threads);
    } else if (threads < 64 || threads > 256 || threads % 64) {
        return fail(NSA_EINVAL, "block_threads %d not a multiple of 64 in [64, 256]", threads);
    }
    if (!(rho > 0.0) || !std::isfinite(rho) || !(mu >= 0.0) || !std::isfinite(mu) || !(dt > 0.0) ||
        !std::isfinite(dt))
        return fail(NSA_EINVAL, "need rho > 0, mu >= 0, dt > 0 (finite); got %g %g %g", rho, mu, dt);
    if ((m->nelem > 0 && !vel) || (m->nnzb > 0 && !values) || (m->npoin > 0 && !rhs))
        return fail(NSA_EINVAL, "nsa_assemble: null device array");
    if (((uintptr_t)values | (uintptr_t)rhs) % 16)
        return fail(NSA_EINVAL, "values and rhs must be 16-byte aligned");
    int dev = -1;
    nsa_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st) return st;
    if (dev != m->device)
        return fail(NSA_EINVAL, "mesh uploaded on device %d, current device is %d", m->device, dev);
    hipStream_t s = (hipStream_t)stream;
    const bool mixed = o.precision == NSA_MIXED;
    if (o.kernel == NSA_KERNEL_GATHER) {
        nsa::GatherArgs a;
        a.ntiles = G.ntiles();
        a.lds_bytes = G.lds[mixed ? 1 : 0];
        a.tile_row = (const int32_t *)(m->ws + G.r_row.off);
        a.tile_nptr = (const int64_t *)(m->ws + G.r_nptr.off);
        a.tile_nodes = (const int32_t *)(m->ws + G.r_nodes.off);
        a.tile_eptr = (const int64_t *)(m->ws + G.r_eptr.off);
        a.rec = (const uint2 *)(m->ws + G.r_recs.off);
        a.tile_pptr = (const int64_t *)(m->ws + G.r_pptr.off);
        a.pairs = (const uint16_t *)(m->ws + G.r_pairs.off);
        a.slot = (const uint32_t *)(m->ws + G.r_slots.off);
        a.bptr = (const int64_t *)(m->ws + m->r_bptr.off);
        a.coord = (const double4 *)(m->ws + m->r_coord4.off);
        a.vel = vel;
        a.vel_soa = vsoa;
        a.rho = rho;
        a.mu = mu;
        a.dt = dt;
        a.accumulate = o.accumulate;
        a.threads = o.block_threads ? o.block_threads : G.threads;
        a.values = values;
        a.rhs = rhs;
        st = hip_check(nsa::launch_gather(mixed ? nsa::TileKern::Mixed : nsa::TileKern::F64, a, s),
                       "assemble (gather)");
        return st ? st : ok();
    }
    if (o.kernel != NSA_KERNEL_DIRECT && P.ok) {
        nsa::TileArgs t;
        t.ntiles = P.ntiles();
        t.lds_bytes = P.lds;
        t.tile_row = (const int32_t *)(m->ws + P.r_row.off);
        t.tile_rptr = (const int64_t *)(m->ws + P.r_rptr.off);
        t.runs = (const uint4 *)(m->ws + P.r_runs.off);
        t.tile_nptr = (const int64_t *)(m->ws + P.r_nptr.off);
        t.tile_nodes = (const int32_t *)(m->ws + P.r_nodes.off);
        t.tile_b0 = (const int64_t *)(m->ws + P.r_b0.off);
        t.tile_npad = (const int32_t *)(m->ws + P.r_npad.off);
        t.cap_nodes = P.cap_nodes;
        t.bptr = (const int64_t *)(m->ws + m->r_bptr.off);
        t.coord = (const double4 *)(m->ws + m->r_coord4.off);
        t.vel = vel;
        t.vel_soa = vsoa;
        t.rho = rho;
        t.mu = mu;
        t.dt = dt;
        t.accumulate = o.accumulate;
        // the deterministic plan relies on one wavefront per tile; the throughput plan accepts a
        // workgroup-size override for tuning
        t.threads = (o.scatter == NSA_COLOUR || o.block_threads == 0) ? P.threads : o.block_threads;
        t.values = values;
        t.rhs = rhs;
        st = hip_check(nsa::launch_tiled(mixed ? nsa::TileKern::Mixed : nsa::TileKern::F64, t, s), "assemble (tiled)");
        return st ? st : ok();
    }
    if (!m->keep_direct)
        return fail(NSA_EUNSUPPORTED, "the direct kernel's data of this mesh was not uploaded (nsa_mesh_keep_direct)");
    if (!o.accumulate) {
        st = hip_check(nsa::launch_fill_zero(values, 16 * m->nnzb, s), "zero values");
        if (st) return st;
        st = hip_check(nsa::launch_fill_zero(rhs, 4 * m->npoin, s), "zero rhs");
        if (st) return st;
    }
    if (m->nelem == 0) return ok();
    nsa::AsmArgs a;
    a.ld = m->nelem;
    a.npoin = m->npoin;
    a.coord = (const double *)(m->ws + m->r_coord.off);
    a.vel = vel;
    a.vel_soa = vsoa;
    a.rho = rho;
    a.mu = mu;
    a.dt = dt;
    a.values = values;
    a.rhs = rhs;
    if (o.scatter == NSA_ATOMIC) {
        a.ln = (const int32_t *)(m->ws + m->r_ln.off);
        a.emap = (const int32_t *)(m->ws + m->r_emap.off);
        a.e0 = 0;
        a.e1 = m->nelem;
        st = hip_check(nsa::launch_assemble(mixed ? nsa::Kern::AtomicMixed : nsa::Kern::AtomicF64, a,
                                            threads, s),
                       "assemble (atomic)");
        if (st) return st;
    } else {
        a.ln = (const int32_t *)(m->ws + m->r_ln_c.off);
        a.emap = (const int32_t *)(m->ws + m->r_emap_c.off);
        for (int c = 0; c < m->ncolours; c++) {
            a.e0 = m->colour_ptr[c];
            a.e1 = m->colour_ptr[c + 1];
            st = hip_check(nsa::launch_assemble(mixed ? nsa::Kern::ColourMixed : nsa::Kern::ColourF64,
                                                a, threads, s),
                           "assemble (colour)");
            if (st) return st;
        }
    }
    return ok();
}

// The err_out report: the sampled elements in the call's precision and in FP64 (see nsa_options).
nsa_status error_report(const nsa_mesh *m, const double *vel, int64_t vel_soa, double rho, double mu, double dt,
                        bool mixed, double *err, hipStream_t s) {
    nsa_status st = hip_check(nsa::launch_fill_zero(err, 12, s), "err_out clear");
    if (st) return st;
    const int64_t ns = std::min<int64_t>(m->nelem, NSA_ERR_SAMPLE);
    if (ns == 0) return ok();
    return hip_check(nsa::launch_err_sample((const int4 *)(m->ws + m->r_esamp.off), (int)ns,
                                            (const double4 *)(m->ws + m->r_coord4.off), vel, vel_soa, rho, mu, rho / dt,
                                            mixed, err, s),
                     "err_out sample");
}
}  // namespace

nsa_status nsa_assemble(const nsa_mesh *m, const double *vel, double rho, double mu, double dt,
                        const nsa_options *opt, double *values, double *rhs, void *stream) {
    nsa_status st = assemble_impl(m, vel, rho, mu, dt, opt, values, rhs, stream);
    if (st || !opt || !opt->err_out) return st;
    st = error_report(m, vel, opt->vel_layout == NSA_VEL_SOA ? m->npoin : 0, rho, mu, dt, opt->precision == NSA_MIXED,
                      opt->err_out, (hipStream_t)stream);
    return st ? st : ok();
}

// ---- batched form ----------------------------------------------------------------------------

}  // extern "C"

struct nsa_batch {
    int32_t scatter = 0;
    // capacity (fixed at creation) and current members
    int32_t cap_meshes = 0;
    int64_t cap_tiles = 0;
    std::vector<const nsa_mesh *> meshes;
    int64_t ntiles = 0;
    int64_t lds = 0;
    int32_t threads = 256;
    int32_t ncu = 256;
    int64_t elements = 0;
    int device = -1;
    nsa::Region r_work, r_desc;
    size_t ws_bytes = 0;
    char *ws = nullptr;
    // pinned host staging: descriptors [cap_meshes] then the work table [cap_tiles] of (mesh, tile)
    char *staging = nullptr;
    size_t staging_desc = 0;             // byte offset of the work table in staging
    hipEvent_t copied = nullptr;         // completion of the last upload from staging
    bool work_dirty = false;             // work table changed since it was last copied
    bool inputs_set = false;
    nsa::TileArgs *desc_host() { return (nsa::TileArgs *)staging; }
    int2 *work_host() { return (int2 *)(staging + staging_desc); }
    ~nsa_batch() {
        // errors cannot be reported from a destructor; the handles are released either way
        if (copied) {
            (void)hipEventSynchronize(copied);
            (void)hipEventDestroy(copied);
        }
        if (staging) (void)hipHostFree(staging);
    }
};

namespace {

nsa_status check_members(int32_t nmesh, const nsa_mesh *const *meshes, int32_t scatter, int64_t *tiles, int *dev,
                         int32_t *threads) {
    for (int32_t i = 0; i < nmesh; i++)
        if (meshes[i] && meshes[i]->family == NSA_QUAD4)
            return fail(NSA_EUNSUPPORTED, "the batched forms take tetrahedral meshes only (member %d)", i);
    *tiles = 0;
    *dev = -1;
    *threads = 0;
    for (int32_t i = 0; i < nmesh; i++) {
        const nsa_mesh *m = meshes[i];
        if (!m) return fail(NSA_EINVAL, "mesh %d is null", i);
        if (!m->ws) return fail(NSA_ESTATE, "mesh %d is not uploaded", i);
        const nsa::TilePlan &P = m->plan[scatter];
        if (!P.ok && m->nelem > 0) return fail(NSA_EUNSUPPORTED, "mesh %d cannot use the tiled kernel", i);
        if (i == 0) *dev = m->device;
        if (m->device != *dev) return fail(NSA_EINVAL, "meshes are on different devices");
        if (P.ok) {
            if (*threads && P.threads != *threads)
                return fail(NSA_EUNSUPPORTED, "meshes planned for different workgroup sizes");
            *threads = P.threads;
        }
        *tiles += P.ntiles();
    }
    return NSA_OK;
}

nsa_status batch_alloc(int32_t cap_meshes, int64_t cap_tiles, int32_t scatter, int dev, nsa_batch **out) {
    nsa_batch *b = nullptr;
    try {
        b = new nsa_batch;
        b->scatter = scatter;
        b->device = dev;
        b->cap_meshes = cap_meshes;
        b->cap_tiles = cap_tiles;
        b->r_desc.off = 0;
        b->r_desc.bytes = (size_t)cap_meshes * sizeof(nsa::TileArgs);
        b->r_work.off = align_up(b->r_desc.bytes);
        b->r_work.bytes = std::max<size_t>(1, (size_t)cap_tiles) * sizeof(int2);
        b->ws_bytes = align_up(b->r_work.off + b->r_work.bytes);
        b->staging_desc = b->r_work.off;
        nsa_status st = hip_check(hipHostMalloc((void **)&b->staging, b->ws_bytes, hipHostMallocDefault),
                                  "hipHostMalloc");
        if (!st) st = hip_check(hipEventCreateWithFlags(&b->copied, hipEventDisableTiming), "hipEventCreate");
        if (!st && dev < 0) st = hip_check(hipGetDevice(&b->device), "hipGetDevice");
        if (!st) st = hip_check(hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, b->device),
                                "hipDeviceGetAttribute");
        if (st) {
            delete b;
            return st;
        }
    } catch (const std::bad_alloc &) {
        delete b;
        return fail(NSA_ENOMEM, "batch: host allocation failed");
    }
    *out = b;
    return NSA_OK;
}

// Install new members (already checked) and write their work table into the staging buffer.
nsa_status batch_fill(nsa_batch *b, int32_t nmesh, const nsa_mesh *const *meshes, int32_t threads) {
    // the staging buffer may still feed the previous upload
    nsa_status st = hip_check(hipEventSynchronize(b->copied), "batch staging wait");
    if (st) return st;
    b->meshes.assign(meshes, meshes + nmesh);
    b->threads = threads ? threads : kPlanThreads[b->scatter];
    b->lds = 0;
    b->elements = 0;
    int2 *w = b->work_host();
    int64_t n = 0;
    for (int32_t i = 0; i < nmesh; i++) {
        const nsa::TilePlan &P = meshes[i]->plan[b->scatter];
        b->lds = std::max<int64_t>(b->lds, P.lds);
        b->elements += meshes[i]->nelem;
        for (int64_t t = 0; t < P.ntiles(); t++) w[n++] = make_int2(i, (int)t);
    }
    b->ntiles = n;
    b->work_dirty = true;
    b->inputs_set = false;
    return NSA_OK;
}

// Copy the work table (if it changed) from staging into the workspace, stream-ordered.
nsa_status batch_push_work(nsa_batch *b, hipStream_t s) {
    if (!b->work_dirty) return NSA_OK;
    if (b->ntiles > 0) {
        nsa_status st = hip_check(hipMemcpyAsync(b->ws + b->r_work.off, b->work_host(), (size_t)b->ntiles * sizeof(int2),
                                                 hipMemcpyHostToDevice, s), "batch work upload");
        if (!st) st = hip_check(hipEventRecord(b->copied, s), "batch event");
        if (st) return st;
    }
    b->work_dirty = false;
    return NSA_OK;
}

// Check member i's inputs and outputs and fill its descriptor (the batched form and its
// allocation-free variant).
nsa_status member_desc(const nsa_mesh *m, int32_t scatter, int32_t i, const double *vel, bool vel_soa, double rho,
                       double mu, double dt, double *values, double *rhs, int32_t accumulate, int32_t threads,
                       nsa::TileArgs &t) {
    const nsa::TilePlan &P = m->plan[scatter];
    if (!(rho > 0.0) || !std::isfinite(rho) || !(mu >= 0.0) || !std::isfinite(mu) || !(dt > 0.0) || !std::isfinite(dt))
        return fail(NSA_EINVAL, "mesh %d: need rho > 0, mu >= 0, dt > 0 (finite)", i);
    if ((m->nelem > 0 && !vel) || (m->nnzb > 0 && !values) || (m->npoin > 0 && !rhs))
        return fail(NSA_EINVAL, "mesh %d: null device array", i);
    if (((uintptr_t)values | (uintptr_t)rhs) % 16) return fail(NSA_EINVAL, "mesh %d: misaligned output", i);
    t = nsa::TileArgs{};
    if (P.ok) {
        t.ntiles = P.ntiles();
        t.lds_bytes = P.lds;
        t.tile_row = (const int32_t *)(m->ws + P.r_row.off);
        t.tile_rptr = (const int64_t *)(m->ws + P.r_rptr.off);
        t.runs = (const uint4 *)(m->ws + P.r_runs.off);
        t.tile_nptr = (const int64_t *)(m->ws + P.r_nptr.off);
        t.tile_nodes = (const int32_t *)(m->ws + P.r_nodes.off);
        t.tile_b0 = (const int64_t *)(m->ws + P.r_b0.off);
        t.tile_npad = (const int32_t *)(m->ws + P.r_npad.off);
        t.cap_nodes = P.cap_nodes;
        t.bptr = (const int64_t *)(m->ws + m->r_bptr.off);
        t.coord = (const double4 *)(m->ws + m->r_coord4.off);
    }
    t.vel = vel;
    t.vel_soa = vel_soa ? m->npoin : 0;
    t.rho = rho;
    t.mu = mu;
    t.dt = dt;
    t.accumulate = accumulate;
    t.threads = threads;
    t.values = values;
    t.rhs = rhs;
    return NSA_OK;
}

}  // namespace

extern "C" {

nsa_status nsa_batch_create(int32_t nmesh, const nsa_mesh *const *meshes, int32_t scatter, nsa_batch **out) {
    if (!out || nmesh <= 0 || !meshes) return fail(NSA_EINVAL, "nsa_batch_create: bad arguments");
    if (scatter != NSA_ATOMIC && scatter != NSA_COLOUR) return fail(NSA_EINVAL, "unknown scatter mode %d", scatter);
    *out = nullptr;
    int64_t tiles = 0;
    int dev = -1;
    int32_t threads = 0;
    nsa_status st = check_members(nmesh, meshes, scatter, &tiles, &dev, &threads);
    if (st) return st;
    if (tiles > (int64_t)INT32_MAX) return fail(NSA_EUNSUPPORTED, "too many tiles in one batch");
    nsa_batch *b = nullptr;
    st = batch_alloc(nmesh, tiles, scatter, dev, &b);
    if (st) return st;
    st = batch_fill(b, nmesh, meshes, threads);
    if (st) {
        delete b;
        return st;
    }
    *out = b;
    return ok();
}

nsa_status nsa_batch_reserve(int32_t max_meshes, int64_t max_tiles, int32_t scatter, nsa_batch **out) {
    if (!out || max_meshes <= 0 || max_tiles <= 0) return fail(NSA_EINVAL, "nsa_batch_reserve: bad arguments");
    if (scatter != NSA_ATOMIC && scatter != NSA_COLOUR) return fail(NSA_EINVAL, "unknown scatter mode %d", scatter);
    if (max_tiles > (int64_t)INT32_MAX) return fail(NSA_EUNSUPPORTED, "too many tiles in one batch");
    *out = nullptr;
    nsa_batch *b = nullptr;
    nsa_status st = batch_alloc(max_meshes, max_tiles, scatter, -1, &b);
    if (st) return st;
    *out = b;
    return ok();
}

nsa_status nsa_batch_reset(nsa_batch *b, int32_t nmesh, const nsa_mesh *const *meshes) {
    if (!b || nmesh <= 0 || !meshes) return fail(NSA_EINVAL, "nsa_batch_reset: bad arguments");
    if (nmesh > b->cap_meshes) return fail(NSA_ENOMEM, "%d meshes, capacity %d", nmesh, b->cap_meshes);
    int64_t tiles = 0;
    int dev = -1;
    int32_t threads = 0;
    nsa_status st = check_members(nmesh, meshes, b->scatter, &tiles, &dev, &threads);
    if (st) return st;
    if (dev != b->device) return fail(NSA_EINVAL, "meshes live on device %d, the batch on %d", dev, b->device);
    if (tiles > b->cap_tiles) return fail(NSA_ENOMEM, "%lld tiles, capacity %lld", (long long)tiles, (long long)b->cap_tiles);
    st = batch_fill(b, nmesh, meshes, threads);
    return st ? st : ok();
}

nsa_status nsa_batch_destroy(nsa_batch *b) {
    delete b;
    return ok();
}

nsa_status nsa_batch_get_info(const nsa_batch *b, size_t *ws_bytes, int64_t *ntiles, int64_t *nelem,
                              int32_t *lds_bytes) {
    if (!b) return fail(NSA_EINVAL, "nsa_batch_get_info: null batch");
    if (ws_bytes) *ws_bytes = b->ws_bytes;
    if (ntiles) *ntiles = b->ntiles;
    if (nelem) *nelem = b->elements;
    if (lds_bytes) *lds_bytes = (int32_t)b->lds;
    return ok();
}

nsa_status nsa_batch_upload(nsa_batch *b, void *ws, size_t ws_bytes, void *stream) {
    if (!b || !ws) return fail(NSA_EINVAL, "nsa_batch_upload: null argument");
    if (ws_bytes < b->ws_bytes) return fail(NSA_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, b->ws_bytes);
    if (((uintptr_t)ws) % 256) return fail(NSA_EINVAL, "workspace not 256-byte aligned");
    int dev = -1;
    nsa_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st) return st;
    if (dev != b->device) return fail(NSA_EINVAL, "batch meshes live on device %d, current is %d", b->device, dev);
    b->ws = (char *)ws;
    b->work_dirty = true;
    st = batch_push_work(b, (hipStream_t)stream);
    if (!st) st = hip_check(nsa::prepare_batch(b->threads, (size_t)kMaxTileLds), "batch LDS limit");
    return st ? st : ok();
}

nsa_status nsa_batch_set_inputs(nsa_batch *b, const double *const *vel, const double *rho, const double *mu,
                                const double *dt, double *const *values, double *const *rhs, int32_t accumulate,
                                void *stream) {
    if (!b || !vel || !rho || !mu || !dt || !values || !rhs) return fail(NSA_EINVAL, "nsa_batch_set_inputs: null argument");
    if (!b->ws) return fail(NSA_ESTATE, "nsa_batch_set_inputs before nsa_batch_upload");
    if (b->meshes.empty()) return fail(NSA_ESTATE, "nsa_batch_set_inputs on a batch without members");
    if (accumulate != 0 && accumulate != 1) return fail(NSA_EINVAL, "accumulate must be 0 or 1");
    // the staging buffer may still feed the previous upload
    nsa_status st = hip_check(hipEventSynchronize(b->copied), "batch staging wait");
    if (st) return st;
    for (size_t i = 0; i < b->meshes.size(); i++) {
        st = member_desc(b->meshes[i], b->scatter, (int32_t)i, vel[i], false, rho[i], mu[i], dt[i], values[i], rhs[i],
                         accumulate, b->threads, b->desc_host()[i]);
        if (st) return st;
    }
    hipStream_t s = (hipStream_t)stream;
    st = hip_check(hipMemcpyAsync(b->ws + b->r_desc.off, b->staging, b->meshes.size() * sizeof(nsa::TileArgs),
                                  hipMemcpyHostToDevice, s), "batch descriptor upload");
    if (st) return st;
    if (b->work_dirty) {
        st = batch_push_work(b, s);  // records the event after both copies
        if (st) return st;
    } else {
        st = hip_check(hipEventRecord(b->copied, s), "batch event");
        if (st) return st;
    }
    b->inputs_set = true;
    return ok();
}

nsa_status nsa_assemble_batched(const nsa_batch *b, const nsa_options *opt, int32_t grid_wgs, void *stream) {
    if (!b) return fail(NSA_EINVAL, "nsa_assemble_batched: null batch");
    if (!b->ws || !b->inputs_set) return fail(NSA_ESTATE, "nsa_assemble_batched before upload / set_inputs");
    nsa_options o{};
    if (opt) o = *opt;
    if (o.precision != NSA_FP64 && o.precision != NSA_MIXED) return fail(NSA_EINVAL, "unknown precision %d", o.precision);
    if (o.scatter != b->scatter) return fail(NSA_EINVAL, "batch was built for scatter mode %d", b->scatter);
    if (o.kernel == NSA_KERNEL_DIRECT) return fail(NSA_EUNSUPPORTED, "the batched form uses the tiled kernel");
    if (o.vel_layout != NSA_VEL_AOS && o.vel_layout != NSA_VEL_SOA)
        return fail(NSA_EINVAL, "unknown velocity layout %d", o.vel_layout);
    if (o.vel_layout != NSA_VEL_AOS)
        return fail(NSA_EUNSUPPORTED, "the batch handle takes velocities as [npoin][3] (NSA_VEL_AOS)");
    if (o.err_out) return fail(NSA_EINVAL, "err_out is taken by nsa_assemble only");
    const int64_t total = b->ntiles;
    if (grid_wgs < 0) return fail(NSA_EINVAL, "grid_wgs must be >= 0");
    int dev = -1;
    nsa_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st) return st;
    if (dev != b->device) return fail(NSA_EINVAL, "batch lives on device %d, current is %d", b->device, dev);
    // the throughput plan accepts a workgroup-size override for tuning; the deterministic plan needs
    // one wavefront per tile
    const int threads = (b->scatter == NSA_ATOMIC && (o.block_threads == 128 || o.block_threads == 192 ||
                                                       o.block_threads == 256))
                            ? o.block_threads : b->threads;
    st = hip_check(nsa::launch_tiled_batch(o.precision == NSA_MIXED ? nsa::TileKern::Mixed : nsa::TileKern::F64,
                                           (const nsa::TileArgs *)(b->ws + b->r_desc.off),
                                           (const int2 *)(b->ws + b->r_work.off), total, threads, b->lds,
                                           grid_wgs, (hipStream_t)stream),
                   "assemble (batched)");
    return st ? st : ok();
}

nsa_status nsa_assemble_batched_static(int32_t nmesh, const nsa_mesh *const *meshes, const double *const *vel,
                                       const double *rho, const double *mu, const double *dt, double *const *values,
                                       double *const *rhs, const nsa_options *opt, void *stream) {
    if (nmesh <= 0 || !meshes || !vel || !rho || !mu || !dt || !values || !rhs)
        return fail(NSA_EINVAL, "nsa_assemble_batched_static: null argument or nmesh <= 0");
    if (nmesh > nsa::kStaticMeshes)
        return fail(NSA_EINVAL, "nsa_assemble_batched_static: %d meshes, at most %d", nmesh, nsa::kStaticMeshes);
    nsa_options o{};
    if (opt) o = *opt;
    if (o.precision != NSA_FP64 && o.precision != NSA_MIXED) return fail(NSA_EINVAL, "unknown precision %d", o.precision);
    if (o.scatter != NSA_ATOMIC && o.scatter != NSA_COLOUR) return fail(NSA_EINVAL, "unknown scatter mode %d", o.scatter);
    if (o.kernel == NSA_KERNEL_DIRECT) return fail(NSA_EUNSUPPORTED, "the batched form uses the tiled kernel");
    if (o.accumulate != 0 && o.accumulate != 1) return fail(NSA_EINVAL, "accumulate must be 0 or 1");
    if (o.vel_layout != NSA_VEL_AOS && o.vel_layout != NSA_VEL_SOA)
        return fail(NSA_EINVAL, "unknown velocity layout %d", o.vel_layout);
    if (o.err_out) return fail(NSA_EINVAL, "err_out is taken by nsa_assemble only");
    int64_t total = 0;
    int mdev = -1;
    int32_t plan_threads = 0;
    nsa_status st = check_members(nmesh, meshes, o.scatter, &total, &mdev, &plan_threads);
    if (st) return st;
    if (total > nsa::kStaticTiles)
        return fail(NSA_EINVAL, "nsa_assemble_batched_static: %lld tiles, at most %lld", (long long)total,
                    (long long)nsa::kStaticTiles);
    int dev = -1;
    st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st) return st;
    if (dev != mdev) return fail(NSA_EINVAL, "meshes live on device %d, current is %d", mdev, dev);
    if (!plan_threads) plan_threads = kPlanThreads[o.scatter];
    const int threads = (o.scatter == NSA_ATOMIC && (o.block_threads == 128 || o.block_threads == 192 ||
                                                       o.block_threads == 256))
                            ? o.block_threads : plan_threads;
    char *base = nullptr;
    st = hip_check(nsa::static_scratch(&base), "static scratch address");
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    // descriptors and first tiles, kDescChunk members per launch; then the work table; then the tiles
    nsa::DescChunk c;
    int64_t lds = 0, off = 0;
    for (int32_t i0 = 0; i0 < nmesh; i0 += nsa::kDescChunk) {
        c.first = i0;
        c.count = std::min<int32_t>(nsa::kDescChunk, nmesh - i0);
        for (int32_t j = 0; j < c.count; j++) {
            const int32_t i = i0 + j;
            st = member_desc(meshes[i], o.scatter, i, vel[i], o.vel_layout == NSA_VEL_SOA, rho[i], mu[i], dt[i],
                             values[i], rhs[i], o.accumulate, plan_threads, c.d[j]);
            if (st) return st;
            c.toff[j] = off;
            off += c.d[j].ntiles;
            lds = std::max<int64_t>(lds, meshes[i]->plan[o.scatter].lds);
        }
        c.toff[c.count] = off;
        st = hip_check(nsa::launch_put_desc(base, c, s), "descriptor launch");
        if (st) return st;
    }
    if (off != total) return fail(NSA_EINVAL, "internal: tile count %lld != %lld", (long long)off, (long long)total);
    st = hip_check(nsa::launch_fill_work(base, nmesh, total, s), "work table launch");
    if (!st) st = hip_check(nsa::prepare_batch(threads, (size_t)kMaxTileLds), "batch LDS limit");
    if (!st)
        st = hip_check(nsa::launch_tiled_batch(o.precision == NSA_MIXED ? nsa::TileKern::Mixed : nsa::TileKern::F64,
                                               (const nsa::TileArgs *)base,
                                               (const int2 *)(base + nsa::kStaticWorkOff), total, threads, lds, 0, s),
                       "assemble (batched, static tables)");
    return st ? st : ok();
}


nsa_status nsa_assemble_residual(const nsa_mesh *m, const double *vel, double rho, double mu, double dt,
                                 const nsa_options *opt, double *rhsid, double *dt_rho, double *mass_rho,
                                 void *stream) {
    if (!m) return fail(NSA_EINVAL, "nsa_assemble_residual: null mesh");
    if (m->family == NSA_QUAD4) return fail(NSA_EUNSUPPORTED, "%s is not available for quadrilateral meshes", __func__);
    if (!m->ws) return fail(NSA_ESTATE, "nsa_assemble_residual: mesh not uploaded");
    nsa_options o{};
    if (opt) o = *opt;
    if (o.precision != NSA_FP64 && o.precision != NSA_MIXED)
        return fail(NSA_EINVAL, "unknown precision %d", o.precision);
    if (o.scatter != NSA_ATOMIC) return fail(NSA_EUNSUPPORTED, "the residual path has the atomic scatter mode only");
    if (o.accumulate != 0 && o.accumulate != 1) return fail(NSA_EINVAL, "accumulate must be 0 or 1");
    if (o.kernel != NSA_KERNEL_AUTO && o.kernel != NSA_KERNEL_TILED)
        return fail(NSA_EUNSUPPORTED, "the residual path has the tiled kernel only");
    if (o.block_threads != 0 && o.block_threads != 256) return fail(NSA_EINVAL, "block_threads must be 0 or 256");
    if (o.vel_layout != NSA_VEL_AOS && o.vel_layout != NSA_VEL_SOA)
        return fail(NSA_EINVAL, "unknown velocity layout %d", o.vel_layout);
    if (o.err_out) return fail(NSA_EINVAL, "err_out is taken by nsa_assemble only");
    const nsa::ResPlan &RP = m->rplan;
    if (!RP.ok && m->npoin > 0)
        return fail(NSA_EUNSUPPORTED, "no residual plan (nsa_mesh_set_tiling with NSA_RESIDUAL_PLAN before upload)");
    if (!(rho > 0.0) || !std::isfinite(rho) || !(mu >= 0.0) || !std::isfinite(mu) || !(dt > 0.0) ||
        !std::isfinite(dt))
        return fail(NSA_EINVAL, "need rho > 0, mu >= 0, dt > 0 (finite); got %g %g %g", rho, mu, dt);
    if ((m->nelem > 0 && !vel) || (m->npoin > 0 && (!rhsid || !dt_rho || !mass_rho)))
        return fail(NSA_EINVAL, "nsa_assemble_residual: null device array");
    if (((uintptr_t)rhsid | (uintptr_t)dt_rho | (uintptr_t)mass_rho) % 8)
        return fail(NSA_EINVAL, "outputs must be 8-byte aligned");
    int dev = -1;
    nsa_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st) return st;
    if (dev != m->device) return fail(NSA_EINVAL, "mesh uploaded on device %d, current device is %d", m->device, dev);
    if (m->npoin == 0) return ok();
    nsa::ResArgs a;
    a.ntiles = RP.ntiles();
    a.lds_bytes = RP.lds;
    a.tile_row = (const int32_t *)(m->ws + RP.r_row.off);
    a.tile_eptr = (const int64_t *)(m->ws + RP.r_eptr.off);
    a.rec = (const uint2 *)(m->ws + RP.r_recs.off);
    a.tile_nptr = (const int64_t *)(m->ws + RP.r_nptr.off);
    a.tile_nodes = (const int32_t *)(m->ws + RP.r_nodes.off);
    a.coord = (const double4 *)(m->ws + m->r_coord4.off);
    a.vel = vel;
    a.vel_soa = o.vel_layout == NSA_VEL_SOA ? m->npoin : 0;
    a.rho = rho;
    a.mu = mu;
    a.dt = dt;
    a.accumulate = o.accumulate;
    a.rhsid = rhsid;
    a.dt_rho = dt_rho;
    a.mass_rho = mass_rho;
    if (RP.r_geo.bytes) {
        a.geo = (const double *)(m->ws + RP.r_geo.off);
        a.rgel = (const uint2 *)(m->ws + RP.r_rgel.off);
    }
    st = hip_check(nsa::launch_residual(o.precision == NSA_MIXED ? nsa::TileKern::Mixed : nsa::TileKern::F64, a,
                                        (hipStream_t)stream), "assemble (residual)");
    return st ? st : ok();
}

nsa_status nsa_bandwidth_probe(int32_t kind, const double *src, double *dst, int64_t n, void *stream) {
    if (kind < NSA_PROBE_READ || kind > NSA_PROBE_COPY || n < 0 || (n & 1) || !dst ||
        (kind != NSA_PROBE_WRITE && !src))
        return fail(NSA_EINVAL, "nsa_bandwidth_probe: bad arguments");
    if (((uintptr_t)src | (uintptr_t)dst) % 16) return fail(NSA_EINVAL, "nsa_bandwidth_probe: 16-byte alignment");
    if (kind == NSA_PROBE_COPY && src < dst + n && dst < src + n)
        return fail(NSA_EINVAL, "nsa_bandwidth_probe: src and dst overlap");
    int dev = 0, ncu = 256;
    nsa_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (!st) st = hip_check(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), "attribute");
    if (!st) st = hip_check(nsa::launch_probe(kind, src, dst, n, ncu, (hipStream_t)stream), "probe");
    return st ? st : ok();
}

nsa_status nsa_fill_uniform(double *out, int64_t n, uint64_t seed, double lo, double hi, void *stream) {
    if (n < 0 || (n > 0 && !out)) return fail(NSA_EINVAL, "nsa_fill_uniform: bad arguments");
    if (!std::isfinite(lo) || !std::isfinite(hi) || !(hi >= lo)) return fail(NSA_EINVAL, "need finite lo <= hi");
    if (((uintptr_t)out) % 8) return fail(NSA_EINVAL, "out must be 8-byte aligned");
    nsa_status st = hip_check(nsa::launch_fill_uniform(out, n, seed, lo, hi, (hipStream_t)stream), "fill uniform");
    return st ? st : ok();
}

}  // extern "C"

