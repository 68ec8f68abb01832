// Host side of libnsa: argument checking, validation, the block pattern of the node graph,
// element colouring, the device data layout and the dispatch of the assembly kernels.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <thread>

#include "nsa_internal.h"

namespace {

thread_local std::string g_last_error;

nsa_status fail(nsa_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

nsa_status ok() {
    g_last_error.clear();
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
    std::vector<uint64_t> mask(2 * (size_t)m->npoin, 0);
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
        if (~f0)
            c = __builtin_ctzll(~f0);
        else if (~f1)
            c = 64 + __builtin_ctzll(~f1);
        else
            return fail(NSA_EUNSUPPORTED, "element %lld needs more than 128 colours", (long long)e);
        for (int a = 0; a < 4; a++) mask[2 * (size_t)ln[a] + (c >> 6)] |= 1ull << (c & 63);
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

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

void plan_layout(nsa_mesh *m) {
    size_t off = 0;
    auto take = [&](nsa::Region &r, size_t bytes) {
        r.off = off;
        r.bytes = bytes;
        off = align_up(off + bytes);
    };
    const size_t ne = (size_t)m->nelem, np = (size_t)m->npoin;
    take(m->r_ln, 4 * ne * sizeof(int32_t));
    take(m->r_coord, 3 * np * sizeof(double));
    take(m->r_emap, 16 * ne * sizeof(int32_t));
    take(m->r_ln_c, 4 * ne * sizeof(int32_t));
    take(m->r_emap_c, 16 * ne * sizeof(int32_t));
    m->ws_bytes = std::max<size_t>(off, 256);
}

nsa_status hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) return fail(NSA_EHIP, "%s: %s", what, hipGetErrorString(e));
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

const char *nsa_last_error(void) { return g_last_error.c_str(); }

int32_t nsa_version(void) { return 100; }

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
        if (st) {
            delete m;
            return st;
        }
        plan_layout(m);
    } catch (const std::bad_alloc &) {
        delete m;
        return fail(NSA_ENOMEM, "nsa_mesh_create: host allocation failed");
    }
    *out = m;
    return ok();
}

nsa_status nsa_mesh_destroy(nsa_mesh *m) {
    delete m;
    return ok();
}

nsa_status nsa_mesh_get_info(const nsa_mesh *m, nsa_mesh_info *info) {
    if (!m || !info) return fail(NSA_EINVAL, "nsa_mesh_get_info: null argument");
    info->npoin = m->npoin;
    info->nelem = m->nelem;
    info->nnzb = m->nnzb;
    info->ncolours = m->ncolours;
    info->uploaded = m->ws != nullptr;
    info->ws_bytes = m->ws_bytes;
    info->max_row_blocks = m->max_row_blocks;
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

nsa_status nsa_mesh_get_colouring(const nsa_mesh *m, int32_t *colour_ptr, int32_t *colour_elems) {
    if (!m) return fail(NSA_EINVAL, "nsa_mesh_get_colouring: null mesh");
    if (m->host_released) return fail(NSA_ESTATE, "host copy released");
    if (colour_ptr) std::copy(m->colour_ptr.begin(), m->colour_ptr.end(), colour_ptr);
    if (colour_elems) std::copy(m->colour_elems.begin(), m->colour_elems.end(), colour_elems);
    return ok();
}

nsa_status nsa_mesh_upload(nsa_mesh *m, void *ws, size_t ws_bytes, void *stream) {
    if (!m || !ws) return fail(NSA_EINVAL, "nsa_mesh_upload: null argument");
    if (m->host_released) return fail(NSA_ESTATE, "host copy released");
    if (ws_bytes < m->ws_bytes)
        return fail(NSA_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, m->ws_bytes);
    if (((uintptr_t)ws) % 256) return fail(NSA_EINVAL, "workspace not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    const int64_t ne = m->nelem, np = m->npoin;
    try {
        std::vector<int32_t> ln(4 * ne), em(16 * ne), lnc(4 * ne), emc(16 * ne);
        std::vector<double> co(3 * np);
        parallel_for(ne, [&](int64_t b, int64_t e) {
            for (int64_t i = b; i < e; i++) {
                for (int a = 0; a < 4; a++) ln[a * ne + i] = m->lnods[4 * i + a];
                for (int k = 0; k < 16; k++) em[k * ne + i] = m->emap[16 * i + k];
                int64_t src = m->colour_elems[i];
                for (int a = 0; a < 4; a++) lnc[a * ne + i] = m->lnods[4 * src + a];
                for (int k = 0; k < 16; k++) emc[k * ne + i] = m->emap[16 * src + k];
            }
        });
        for (int64_t i = 0; i < np; i++)
            for (int d = 0; d < 3; d++) co[d * np + i] = m->coord[3 * i + d];
        char *w = (char *)ws;
        nsa_status st;
        struct Up { const nsa::Region &r; const void *src; };
        const Up ups[] = {{m->r_ln, ln.data()}, {m->r_coord, co.data()}, {m->r_emap, em.data()},
                          {m->r_ln_c, lnc.data()}, {m->r_emap_c, emc.data()}};
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
    m->host_released = true;
    return ok();
}

nsa_status nsa_assemble(const nsa_mesh *m, const double *vel, double rho, double mu, double dt,
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
    for (int r : o.reserved)
        if (r) return fail(NSA_EINVAL, "reserved option fields must be zero");
    int threads = o.block_threads ? o.block_threads : 256;
    if (threads < 64 || threads > 256 || threads % 64)
        return fail(NSA_EINVAL, "block_threads %d not a multiple of 64 in [64, 256]", threads);
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
    a.rho = rho;
    a.mu = mu;
    a.dt = dt;
    a.values = values;
    a.rhs = rhs;
    const bool mixed = o.precision == NSA_MIXED;
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

}  // extern "C"
