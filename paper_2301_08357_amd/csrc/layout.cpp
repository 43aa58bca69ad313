// Host-side mesh ingest: validation, orientation, Morton renumbering,
// element ordering, node-to-element lists and Morton tiles.
#include "layout.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace pm {

namespace {

// Spread the low 21 bits of v so that bit b lands on bit 3b (3D) or 2b (2D).
inline uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

inline uint64_t spread2(uint64_t v)
{
    v &= 0x1fffffULL;
    v = (v | (v << 16)) & 0x0000ffff0000ffffULL;
    v = (v | (v << 8)) & 0x00ff00ff00ff00ffULL;
    v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0fULL;
    v = (v | (v << 2)) & 0x3333333333333333ULL;
    v = (v | (v << 1)) & 0x5555555555555555ULL;
    return v;
}

// Component c of the edge vector p_k - p_0, shifted along a periodic axis
// (L > 0, iL = 1/L) by the multiple of L that brings it into [-L/2, L/2].
inline double edge(const double *pk, const double *p0, int c, const double *L, const double *iL)
{
    const double d = pk[c] - p0[c];
    return L[c] > 0.0 ? std::fma(-L[c], std::nearbyint(d * iL[c]), d) : d;
}

// Signed Jacobian determinant of the (minimum-image) edge vectors:
// e1 x e2 in 2D, e1 . (e2 x e3) in 3D.
inline double simplex_det(int dim, const double *c, const int32_t *v, const double *L, const double *iL)
{
    if (dim == 2) {
        const double *p0 = c + 2 * (int64_t)v[0], *p1 = c + 2 * (int64_t)v[1], *p2 = c + 2 * (int64_t)v[2];
        double ax = edge(p1, p0, 0, L, iL), ay = edge(p1, p0, 1, L, iL);
        double bx = edge(p2, p0, 0, L, iL), by = edge(p2, p0, 1, L, iL);
        return ax * by - ay * bx;
    }
    const double *p0 = c + 3 * (int64_t)v[0], *p1 = c + 3 * (int64_t)v[1];
    const double *p2 = c + 3 * (int64_t)v[2], *p3 = c + 3 * (int64_t)v[3];
    double a[3], b[3], d[3];
    for (int k = 0; k < 3; ++k) {
        a[k] = edge(p1, p0, k, L, iL);
        b[k] = edge(p2, p0, k, L, iL);
        d[k] = edge(p3, p0, k, L, iL);
    }
    double cx = b[1] * d[2] - b[2] * d[1];
    double cy = b[2] * d[0] - b[0] * d[2];
    double cz = b[0] * d[1] - b[1] * d[0];
    return a[0] * cx + a[1] * cy + a[2] * cz;
}

}  // namespace

int build_layout(const pm_mesh *m, Layout *L)
{
    if (!m || !L || !m->coords || !m->elems) return PM_EINVAL;
    const int dim = m->dim;
    if (dim != 2 && dim != 3) return PM_EINVAL;
    const int64_t N = m->n_nodes, E = m->n_elems;
    if (N < 1 || N >= INT32_MAX || E < 1 || E >= (int64_t(1) << 29)) return PM_EINVAL;
    const int nv = dim + 1;
    for (int64_t i = 0; i < N * dim; ++i)
        if (!std::isfinite(m->coords[i])) return PM_EINVAL;
    double per[3] = {0.0, 0.0, 0.0}, iper[3] = {0.0, 0.0, 0.0};
    L->periodic = false;
    if (m->period)
        for (int ax = 0; ax < dim; ++ax) {
            const double p = m->period[ax];
            if (!std::isfinite(p) || p < 0.0) return PM_EINVAL;
            if (p > 0.0) {
                per[ax] = p;
                iper[ax] = 1.0 / p;
                L->periodic = true;
            }
        }
    for (int ax = 0; ax < 3; ++ax) L->period[ax] = per[ax];

    // 1. indices and orientation
    std::vector<int32_t> el(m->elems, m->elems + E * nv);
    for (int64_t e = 0; e < E; ++e) {
        int32_t *v = el.data() + e * nv;
        for (int a = 0; a < nv; ++a)
            if (v[a] < 0 || v[a] >= N) return PM_EINVAL;
        double det = simplex_det(dim, m->coords, v, per, iper);
        if (det == 0.0 || !std::isfinite(det)) return PM_EDEGENERATE;
        if (det < 0.0) std::swap(v[1], v[2]);
    }

    // 2. Morton keys and node order (key, old id)
    std::vector<uint64_t> key(N);
    if (m->lattice) {
        for (int64_t i = 0; i < N; ++i) {
            uint64_t k = 0;
            for (int ax = 0; ax < dim; ++ax) {
                int32_t q = m->lattice[i * dim + ax];
                if (q < 0 || q > 2097151) return PM_EINVAL;
                k |= (dim == 3 ? spread3(uint64_t(q)) : spread2(uint64_t(q))) << ax;
            }
            key[i] = k;
        }
    } else {
        double lo[3], hi[3];
        for (int ax = 0; ax < dim; ++ax) { lo[ax] = INFINITY; hi[ax] = -INFINITY; }
        for (int64_t i = 0; i < N; ++i)
            for (int ax = 0; ax < dim; ++ax) {
                double v = m->coords[i * dim + ax];
                lo[ax] = std::min(lo[ax], v);
                hi[ax] = std::max(hi[ax], v);
            }
        for (int64_t i = 0; i < N; ++i) {
            uint64_t k = 0;
            for (int ax = 0; ax < dim; ++ax) {
                uint64_t q = 0;
                if (hi[ax] > lo[ax]) {
                    volatile double t = (m->coords[i * dim + ax] - lo[ax]) / (hi[ax] - lo[ax]);
                    q = uint64_t(std::floor(t * 2097151.0));
                }
                k |= (dim == 3 ? spread3(q) : spread2(q)) << ax;
            }
            key[i] = k;
        }
    }
    std::vector<int32_t> order(N);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return key[a] != key[b] ? key[a] < key[b] : a < b;
    });
    std::vector<int32_t> old2new(N);
    for (int64_t r = 0; r < N; ++r) old2new[order[r]] = int32_t(r);

    // 3. element order: stable counting sort by smallest new vertex
    std::vector<int32_t> emin(E);
    std::vector<int64_t> cnt(N + 1, 0);
    for (int64_t e = 0; e < E; ++e) {
        int32_t mn = INT32_MAX;
        for (int a = 0; a < nv; ++a) mn = std::min(mn, old2new[el[e * nv + a]]);
        emin[e] = mn;
        cnt[mn + 1]++;
    }
    for (int64_t i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
    L->elem_new2old.assign(E, 0);
    for (int64_t e = 0; e < E; ++e) L->elem_new2old[cnt[emin[e]]++] = int32_t(e);

    // 4. connectivity in internal numbering and node-to-element lists
    L->dim = dim;
    L->n_nodes = N;
    L->n_elems = E;
    L->node_new2old = std::move(order);
    L->conn.assign(E * 4, 0);
    L->n2e_off.assign(N + 1, 0);
    for (int64_t r = 0; r < E; ++r) {
        const int32_t *v = el.data() + int64_t(L->elem_new2old[r]) * nv;
        for (int a = 0; a < nv; ++a) {
            int32_t w = old2new[v[a]];
            L->conn[r * 4 + a] = w;
            L->n2e_off[w + 1]++;
        }
    }
    for (int64_t i = 0; i < N; ++i) L->n2e_off[i + 1] += L->n2e_off[i];
    L->n2e_ent.assign(E * nv, 0);
    {
        std::vector<int32_t> fill(L->n2e_off.begin(), L->n2e_off.end() - 1);
        for (int64_t r = 0; r < E; ++r)
            for (int a = 0; a < nv; ++a) {
                int32_t w = L->conn[r * 4 + a];
                L->n2e_ent[fill[w]++] = int32_t(4 * r + a);
            }
    }

    // 5. node data in internal order
    L->dirichlet.assign(N, 0);
    L->coords.assign(N * dim, 0.0);
    int64_t nfree = 0;
    for (int64_t r = 0; r < N; ++r) {
        int32_t o = L->node_new2old[r];
        uint8_t d = (m->dirichlet && m->dirichlet[o]) ? 1 : 0;
        L->dirichlet[r] = d;
        nfree += !d;
        for (int ax = 0; ax < dim; ++ax) L->coords[ax * N + r] = m->coords[int64_t(o) * dim + ax];
    }
    L->n_free = nfree;
    return PM_OK;
}

int build_tiles(const Layout &L, int tile_nodes, Tiles *T, int64_t n_tiles)
{
    const int64_t N = L.n_nodes, E = L.n_elems;
    const int nv = L.dim + 1;
    if (tile_nodes < 64 || tile_nodes > 4096) return PM_EINVAL;
    if (n_tiles < 0 || n_tiles > N || (n_tiles > 0 && (N + n_tiles - 1) / n_tiles > tile_nodes)) return PM_EINVAL;
    T->tile_nodes = tile_nodes;
    T->n_tiles = n_tiles > 0 ? n_tiles : (N + tile_nodes - 1) / tile_nodes;
    const int64_t nt = T->n_tiles;
    T->node_off.assign(nt + 1, 0);
    for (int64_t t = 0; t <= nt; ++t)
        T->node_off[t] = int32_t(n_tiles > 0 ? (t * N) / nt : std::min<int64_t>(N, t * tile_nodes));
    T->halo_off.assign(nt + 1, 0);
    T->inst_off.assign(nt + 1, 0);
    T->halo.clear();
    T->inst_elem.clear();
    T->inst.clear();
    T->inst_elem.reserve(size_t(E) * 3 / 2 + 16);
    T->inst.reserve(size_t(E) * 6 + 64);
    T->lvb = (tile_nodes <= 256) ? 10 : 11;
    const int max_rows = 1 << (16 - T->lvb), max_local = 1 << T->lvb;
    T->max_inst = 0;
    T->max_halo = 0;
    T->max_deg = 0;
    for (int64_t i = 0; i < N; ++i) T->max_deg = std::max<int>(T->max_deg, L.n2e_off[i + 1] - L.n2e_off[i]);
    if (T->max_deg >= max_rows) return TILES_TOO_WIDE;   // row max_deg takes the halo vertices

    // first element whose smallest vertex is >= v (elements are sorted by it)
    std::vector<int32_t> ebeg(N + 1, 0);
    for (int64_t e = 0; e < E; ++e) {
        int32_t mn = INT32_MAX;
        for (int a = 0; a < nv; ++a) mn = std::min(mn, L.conn[e * 4 + a]);
        ebeg[mn + 1]++;
    }
    for (int64_t i = 0; i < N; ++i) ebeg[i + 1] += ebeg[i];

    std::vector<int32_t> halo_el, halo_nd;
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t s = T->node_off[t], f = T->node_off[t + 1];
        const int32_t own0 = ebeg[s], own1 = ebeg[f];
        halo_el.clear();
        for (int64_t i = s; i < f; ++i)
            for (int32_t k = L.n2e_off[i]; k < L.n2e_off[i + 1]; ++k) {
                int32_t e = L.n2e_ent[k] >> 2;
                if (e < own0) halo_el.push_back(e);
            }
        std::sort(halo_el.begin(), halo_el.end());
        halo_el.erase(std::unique(halo_el.begin(), halo_el.end()), halo_el.end());
        const int64_t ninst = int64_t(halo_el.size()) + (own1 - own0);
        // halo nodes: vertices of the instances outside [s, f)
        halo_nd.clear();
        auto add_halo = [&](int32_t e) {
            for (int a = 0; a < nv; ++a) {
                int32_t v = L.conn[e * 4 + a];
                if (v < s || v >= f) halo_nd.push_back(v);
            }
        };
        for (int32_t e : halo_el) add_halo(e);
        for (int32_t e = own0; e < own1; ++e) add_halo(e);
        std::sort(halo_nd.begin(), halo_nd.end());
        halo_nd.erase(std::unique(halo_nd.begin(), halo_nd.end()), halo_nd.end());
        if (int64_t(tile_nodes) + int64_t(halo_nd.size()) > max_local) return TILES_TOO_WIDE;
        T->halo.insert(T->halo.end(), halo_nd.begin(), halo_nd.end());
        T->halo_off[t + 1] = int32_t(T->halo.size());
        T->max_halo = std::max<int>(T->max_halo, int(halo_nd.size()));
        auto local = [&](int32_t v) -> uint16_t {
            if (v >= s && v < f) return uint16_t(v - s);
            return uint16_t(tile_nodes + (std::lower_bound(halo_nd.begin(), halo_nd.end(), v) - halo_nd.begin()));
        };
        const size_t base = T->inst_elem.size();
        auto add_inst = [&](int32_t e) {
            T->inst_elem.push_back(e);
            for (int a = 0; a < 4; ++a) {
                uint16_t f = 0;
                if (a < nv) {
                    f = local(L.conn[e * 4 + a]);
                    if (f >= tile_nodes) f = uint16_t(f | (T->max_deg << T->lvb));   // halo vertex: the extra row
                }
                T->inst.push_back(f);
            }
        };
        for (int32_t e : halo_el) add_inst(e);
        for (int32_t e = own0; e < own1; ++e) add_inst(e);
        // rows: node i's incidence list is ascending in element id, and the
        // instance index is ascending in element id too
        for (int64_t i = s; i < f; ++i) {
            int row = 0;
            for (int32_t k = L.n2e_off[i]; k < L.n2e_off[i + 1]; ++k, ++row) {
                int32_t e = L.n2e_ent[k] >> 2, a = L.n2e_ent[k] & 3;
                int32_t li = (e >= own0) ? int32_t(halo_el.size()) + (e - own0)
                                         : int32_t(std::lower_bound(halo_el.begin(), halo_el.end(), e) - halo_el.begin());
                T->inst[(base + li) * 4 + a] |= uint16_t(row << T->lvb);
            }
        }
        T->inst_off[t + 1] = int32_t(T->inst_elem.size());
        T->max_inst = std::max<int>(T->max_inst, int(ninst));
    }
    return PM_OK;
}

int build_faces(const pm_mesh *m, Faces *F)
{
    if (!m || !F || !m->elems) return PM_EINVAL;
    const int dim = m->dim;
    if (dim != 2 && dim != 3) return PM_EINVAL;
    const int64_t N = m->n_nodes, E = m->n_elems;
    const int nv = dim + 1;
    if (N < 1 || E < 1 || E >= (int64_t(1) << 29)) return PM_EINVAL;
    // one record per (element, local vertex): the sorted tuple of the other
    // vertices, then the element, then the local vertex
    struct Rec {
        int32_t v[3];
        int32_t e, a;
    };
    std::vector<Rec> rec(size_t(E) * nv);
    for (int64_t e = 0; e < E; ++e) {
        const int32_t *ev = m->elems + e * nv;
        for (int a = 0; a < nv; ++a) {
            Rec &r = rec[size_t(e) * nv + a];
            int k = 0;
            for (int b = 0; b < nv; ++b) {
                if (b == a) continue;
                if (ev[b] < 0 || ev[b] >= N) return PM_EINVAL;
                r.v[k++] = ev[b];
            }
            if (dim == 2) r.v[2] = -1;
            std::sort(r.v, r.v + dim);
            r.e = int32_t(e);
            r.a = a;
        }
    }
    std::sort(rec.begin(), rec.end(), [](const Rec &x, const Rec &y) {
        if (x.v[0] != y.v[0]) return x.v[0] < y.v[0];
        if (x.v[1] != y.v[1]) return x.v[1] < y.v[1];
        if (x.v[2] != y.v[2]) return x.v[2] < y.v[2];
        return x.e != y.e ? x.e < y.e : x.a < y.a;
    });
    F->dim = dim;
    F->vertices.clear();
    F->elems.clear();
    F->elem_face.assign(size_t(E) * nv, -1);
    int64_t nb = 0;
    for (size_t i = 0; i < rec.size();) {
        size_t j = i + 1;
        while (j < rec.size() && std::equal(rec[j].v, rec[j].v + dim, rec[i].v)) ++j;
        if (j - i > 2) return PM_EINVAL;
        const int32_t f = int32_t(F->vertices.size() / dim);
        F->vertices.insert(F->vertices.end(), rec[i].v, rec[i].v + dim);
        F->elems.push_back(rec[i].e);
        F->elems.push_back(j - i == 2 ? rec[i + 1].e : -1);
        nb += (j - i == 1);
        for (size_t k = i; k < j; ++k) F->elem_face[size_t(rec[k].e) * nv + rec[k].a] = f;
        i = j;
    }
    F->n_faces = int64_t(F->vertices.size() / dim);
    F->n_boundary = nb;
    return PM_OK;
}

}  // namespace pm
