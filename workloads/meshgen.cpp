// Native half of the seeded input generators: the same constructions as the
// Python generators in workloads/__init__.py, written for multi-million-atom
// inputs.  Inputs only: no part of the solver's arithmetic lives here.
//
//   mg_accept_min_sep  -- sequential acceptance of candidate atom positions
//                         that keep a minimum separation (uniform grid hash)
//   mg_density         -- Gaussian density sum_k exp(-beta (|x-r_k|^2/R_k^2 - 1))
//                         on a regular grid, truncated at trunc R_k, every
//                         grid point summed over its atoms in atom order
//   mg_march / mg_march_fetch
//                      -- marching tetrahedra over the Freudenthal split of
//                         the grid cubes (six tetrahedra around the main
//                         diagonal, so the complex is conforming and the
//                         surface closed), vertices on grid edges numbered by
//                         first use in tetrahedron order, interpolation
//                         parameter clamped to [clamp, 1 - clamp], triangles
//                         oriented from inside corners to outside corners.
//
// Built with g++ -O2 -fopenmp -ffp-contract=off (no fused multiply-add, so
// the arithmetic matches the numpy generator operation for operation).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <parallel/algorithm>
#include <unordered_map>
#include <vector>

#include <omp.h>

namespace {

// the six tetrahedra: corner c0 = (0,0,0), then one axis at a time set to 1
// in the order of each permutation of (x, y, z), ending at (1,1,1);
// permutations in lexicographic order
const int KUHN_PERM[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

struct Tet {
    int64_t gid[4];      // grid point ids of the corners
    int cx[4][3];        // corner offsets from the cube's base point
};

void kuhn_tet(int t, int c[4][3]) {
    int cur[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) c[0][d] = 0;
    for (int s = 0; s < 3; ++s) {
        cur[KUHN_PERM[t][s]] = 1;
        for (int d = 0; d < 3; ++d) c[s + 1][d] = cur[d];
    }
}

struct SlabOut {
    // per crossing-edge slot: edge key, inside/outside grid ids, values
    std::vector<int64_t> key, ga, gb;
    std::vector<double> fa, fb;
    // per triangle: three slot indices (local to the slab), owning tet's
    // inside/outside corner centroids (grid units)
    std::vector<int64_t> tri;
    std::vector<double> cin, cout;
};

struct MarchState {
    std::vector<double> V;
    std::vector<int32_t> T;
};
MarchState *g_last = nullptr;

}  // namespace

extern "C" {

// Accepts candidates in order while each is at least min_sep from every
// accepted one; stops after nmax acceptances.  cand [nc][3]; idx receives
// the accepted candidates' indices.  Returns the number accepted.
long mg_accept_min_sep(long nc, const double *cand, double min_sep, long nmax, long *idx) {
    const double cell = min_sep, ms2 = min_sep * min_sep;
    std::unordered_map<int64_t, std::vector<int32_t>> grid;
    grid.reserve((size_t)nmax * 2);
    auto key = [](int64_t a, int64_t b, int64_t c) {
        return ((a + (1 << 20)) << 42) | ((b + (1 << 20)) << 21) | (c + (1 << 20));
    };
    long count = 0;
    std::vector<double> acc;
    acc.reserve((size_t)3 * nmax);
    for (long i = 0; i < nc && count < nmax; ++i) {
        const double *p = cand + 3 * i;
        const int64_t kx = (int64_t)std::floor(p[0] / cell), ky = (int64_t)std::floor(p[1] / cell),
                      kz = (int64_t)std::floor(p[2] / cell);
        bool ok = true;
        for (int dx = -1; dx <= 1 && ok; ++dx)
            for (int dy = -1; dy <= 1 && ok; ++dy)
                for (int dz = -1; dz <= 1 && ok; ++dz) {
                    auto it = grid.find(key(kx + dx, ky + dy, kz + dz));
                    if (it == grid.end()) continue;
                    for (int32_t j : it->second) {
                        const double *q = acc.data() + 3 * (size_t)j;
                        const double ddx = q[0] - p[0], ddy = q[1] - p[1], ddz = q[2] - p[2];
                        if ((ddx * ddx + ddy * ddy) + ddz * ddz < ms2) { ok = false; break; }
                    }
                }
        if (!ok) continue;
        grid[key(kx, ky, kz)].push_back((int32_t)count);
        acc.push_back(p[0]);
        acc.push_back(p[1]);
        acc.push_back(p[2]);
        idx[count++] = i;
    }
    return count;
}

// rho[(i ny + j) nz + k] = sum over atoms (in order) of
// exp(-beta (d2 / R^2 - 1)) for d2 <= (trunc R)^2, with d2 = (dx^2 + dy^2)
// + dz^2 and grid coordinates lo + h i.
int mg_density(long na, const double *atoms, const double *radii, const double *lo, double h,
               long nx, long ny, long nz, double beta, double trunc, double *rho) {
    // atoms binned by the x-planes they reach, in atom order
    std::vector<long> cnt(nx + 1, 0);
    std::vector<long> i0v(na), i1v(na);
    for (long a = 0; a < na; ++a) {
        const double rc = trunc * radii[a];
        long i0 = (long)std::floor((atoms[3 * a] - rc - lo[0]) / h);
        long i1 = (long)std::ceil((atoms[3 * a] + rc - lo[0]) / h) + 1;
        i0 = std::max(0l, i0);
        i1 = std::min(nx, i1);
        i0v[a] = i0;
        i1v[a] = i1;
        for (long i = i0; i < i1; ++i) ++cnt[i + 1];
    }
    for (long i = 0; i < nx; ++i) cnt[i + 1] += cnt[i];
    std::vector<long> lst(cnt[nx]);
    {
        std::vector<long> fill(cnt.begin(), cnt.end() - 1);
        for (long a = 0; a < na; ++a)
            for (long i = i0v[a]; i < i1v[a]; ++i) lst[fill[i]++] = a;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < nx; ++i) {
        double *plane = rho + (size_t)i * ny * nz;
        std::memset(plane, 0, sizeof(double) * ny * nz);
        const double gx = lo[0] + h * (double)i;
        for (long q = cnt[i]; q < cnt[i + 1]; ++q) {
            const long a = lst[q];
            const double ax = atoms[3 * a], ay = atoms[3 * a + 1], az = atoms[3 * a + 2];
            const double r = radii[a], rc = trunc * r;
            long j0 = std::max(0l, (long)std::floor((ay - rc - lo[1]) / h));
            long j1 = std::min(ny, (long)std::ceil((ay + rc - lo[1]) / h) + 1);
            long k0 = std::max(0l, (long)std::floor((az - rc - lo[2]) / h));
            long k1 = std::min(nz, (long)std::ceil((az + rc - lo[2]) / h) + 1);
            const double dx = gx - ax, dx2 = dx * dx;
            const double inv = 1.0 / (r * r), rc2 = rc * rc;
            for (long j = j0; j < j1; ++j) {
                const double dy = (lo[1] + h * (double)j) - ay, dxy = dx2 + dy * dy;
                double *row = plane + (size_t)j * nz;
                for (long k = k0; k < k1; ++k) {
                    const double dz = (lo[2] + h * (double)k) - az;
                    const double d2 = dxy + dz * dz;
                    if (d2 > rc2) continue;
                    row[k] += std::exp(-beta * (d2 * inv - 1.0));
                }
            }
        }
    }
    return 0;
}

// Marching tetrahedra on F (grid values minus the level; no value may be 0).
// Returns 0 and the vertex / triangle counts; mg_march_fetch copies them.
int mg_march(const double *F, long nx, long ny, long nz, const double *lo, double h,
             double clamp, long *nv_out, long *nt_out) {
    delete g_last;
    g_last = nullptr;
    const int64_t NY = ny, NZ = nz;
    auto gidx = [&](int64_t i, int64_t j, int64_t k) { return (i * NY + j) * NZ + k; };
    const int64_t npts = (int64_t)nx * ny * nz;
    int tetc[6][4][3];
    for (int t = 0; t < 6; ++t) kuhn_tet(t, tetc[t]);
    std::vector<SlabOut> slab(nx > 1 ? nx - 1 : 0);
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < nx - 1; ++i) {
        SlabOut &o = slab[i];
        for (long j = 0; j < ny - 1; ++j)
            for (long k = 0; k < nz - 1; ++k) {
                bool anyin = false, allin = true;
                for (int c = 0; c < 8; ++c) {
                    const bool in = F[gidx(i + (c >> 2), j + ((c >> 1) & 1), k + (c & 1))] > 0.0;
                    anyin |= in;
                    allin &= in;
                }
                if (!anyin || allin) continue;
                for (int t = 0; t < 6; ++t) {
                    int64_t g[4];
                    double v[4];
                    bool ins[4];
                    int nin = 0;
                    for (int c = 0; c < 4; ++c) {
                        g[c] = gidx(i + tetc[t][c][0], j + tetc[t][c][1], k + tetc[t][c][2]);
                        v[c] = F[g[c]];
                        ins[c] = v[c] > 0.0;
                        nin += ins[c];
                    }
                    if (nin == 0 || nin == 4) continue;
                    // inside corners first, then outside, each in corner order
                    int ord[4], q = 0;
                    for (int c = 0; c < 4; ++c) if (ins[c]) ord[q++] = c;
                    for (int c = 0; c < 4; ++c) if (!ins[c]) ord[q++] = c;
                    int ea[4], eb[4], ns;
                    if (nin == 1) {
                        ns = 3;
                        for (int s = 0; s < 3; ++s) { ea[s] = ord[0]; eb[s] = ord[s + 1]; }
                    } else if (nin == 3) {
                        ns = 3;
                        for (int s = 0; s < 3; ++s) { ea[s] = ord[s]; eb[s] = ord[3]; }
                    } else {
                        ns = 4;
                        ea[0] = ord[0]; eb[0] = ord[2];
                        ea[1] = ord[0]; eb[1] = ord[3];
                        ea[2] = ord[1]; eb[2] = ord[3];
                        ea[3] = ord[1]; eb[3] = ord[2];
                    }
                    const int64_t base = (int64_t)o.key.size();
                    for (int s = 0; s < ns; ++s) {
                        const int64_t a = g[ea[s]], b = g[eb[s]];
                        o.key.push_back(std::min(a, b) * npts + std::max(a, b));
                        o.ga.push_back(a);
                        o.gb.push_back(b);
                        o.fa.push_back(v[ea[s]]);
                        o.fb.push_back(v[eb[s]]);
                    }
                    // inside / outside corner centroids in grid units
                    int64_t si[3] = {0, 0, 0}, so[3] = {0, 0, 0};
                    for (int c = 0; c < 4; ++c)
                        for (int d = 0; d < 3; ++d) {
                            const int64_t pc = (d == 0 ? i : d == 1 ? j : k) + tetc[t][c][d];
                            if (ins[c]) si[d] += pc; else so[d] += pc;
                        }
                    double ci[3], co[3];
                    for (int d = 0; d < 3; ++d) {
                        ci[d] = (double)si[d] / (double)nin;
                        co[d] = (double)so[d] / (double)(4 - nin);
                    }
                    auto emit = [&](int s0, int s1, int s2) {
                        o.tri.push_back(base + s0);
                        o.tri.push_back(base + s1);
                        o.tri.push_back(base + s2);
                        for (int d = 0; d < 3; ++d) { o.cin.push_back(ci[d]); o.cout.push_back(co[d]); }
                    };
                    emit(0, 1, 2);
                    if (nin == 2) emit(0, 2, 3);
                }
            }
    }
    // global slot and triangle numbering in slab order
    const long ns_slab = (long)slab.size();
    std::vector<int64_t> soff(ns_slab + 1, 0), toff(ns_slab + 1, 0);
    for (long s = 0; s < ns_slab; ++s) {
        soff[s + 1] = soff[s] + (int64_t)slab[s].key.size();
        toff[s + 1] = toff[s] + (int64_t)slab[s].tri.size() / 3;
    }
    const int64_t nslot = soff[ns_slab], ntri = toff[ns_slab];
    // (key, slot) sorted: the first slot of each key defines its vertex
    std::vector<std::pair<int64_t, int64_t>> ks(nslot);
#pragma omp parallel for schedule(dynamic, 1)
    for (long s = 0; s < ns_slab; ++s)
        for (size_t q = 0; q < slab[s].key.size(); ++q)
            ks[soff[s] + q] = {slab[s].key[q], soff[s] + (int64_t)q};
    __gnu_parallel::sort(ks.begin(), ks.end());
    std::vector<int64_t> defslot;
    defslot.reserve(nslot / 4 + 1);
    for (int64_t q = 0; q < nslot; ++q)
        if (q == 0 || ks[q].first != ks[q - 1].first) defslot.push_back(ks[q].second);
    const int64_t nv = (int64_t)defslot.size();
    // vertices numbered by first appearance
    std::vector<int64_t> byfirst(defslot);
    __gnu_parallel::sort(byfirst.begin(), byfirst.end());
    std::vector<int64_t> slot_vid(nslot, -1);
    {
        // rank of each defining slot, then propagated along its key's run
        std::vector<int64_t> rank_of_run(nv);
#pragma omp parallel for
        for (int64_t r = 0; r < nv; ++r) {
            const int64_t pos = std::lower_bound(byfirst.begin(), byfirst.end(), defslot[r]) - byfirst.begin();
            rank_of_run[r] = pos;
        }
        int64_t run = -1;
        for (int64_t q = 0; q < nslot; ++q) {
            if (q == 0 || ks[q].first != ks[q - 1].first) ++run;
            slot_vid[ks[q].second] = rank_of_run[run];
        }
    }
    auto *res = new MarchState();
    res->V.resize((size_t)3 * nv);
    auto slot_ref = [&](int64_t gs, long &s, int64_t &loc) {
        s = (long)(std::upper_bound(soff.begin(), soff.end(), gs) - soff.begin()) - 1;
        loc = gs - soff[s];
    };
#pragma omp parallel for
    for (int64_t vtx = 0; vtx < nv; ++vtx) {
        long s;
        int64_t loc;
        slot_ref(byfirst[vtx], s, loc);
        const SlabOut &o = slab[s];
        double t = o.fa[loc] / (o.fa[loc] - o.fb[loc]);
        t = std::min(1.0 - clamp, std::max(clamp, t));
        const int64_t a = o.ga[loc], b = o.gb[loc];
        const int64_t pa[3] = {a / (NY * NZ), (a / NZ) % NY, a % NZ};
        const int64_t pb[3] = {b / (NY * NZ), (b / NZ) % NY, b % NZ};
        for (int d = 0; d < 3; ++d) {
            const double fa = (double)pa[d], fb = (double)pb[d];
            res->V[3 * vtx + d] = lo[d] + h * (fa + t * (fb - fa));
        }
    }
    res->T.resize((size_t)3 * ntri);
#pragma omp parallel for schedule(dynamic, 1)
    for (long s = 0; s < ns_slab; ++s) {
        const SlabOut &o = slab[s];
        const int64_t nt = (int64_t)o.tri.size() / 3;
        for (int64_t q = 0; q < nt; ++q) {
            int64_t v0 = slot_vid[soff[s] + o.tri[3 * q]], v1 = slot_vid[soff[s] + o.tri[3 * q + 1]],
                    v2 = slot_vid[soff[s] + o.tri[3 * q + 2]];
            const double *P0 = &res->V[3 * v0], *P1 = &res->V[3 * v1], *P2 = &res->V[3 * v2];
            const double e1[3] = {P1[0] - P0[0], P1[1] - P0[1], P1[2] - P0[2]};
            const double e2[3] = {P2[0] - P0[0], P2[1] - P0[1], P2[2] - P0[2]};
            const double nrm[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                                   e1[0] * e2[1] - e1[1] * e2[0]};
            const double *ci = &o.cin[3 * q], *co = &o.cout[3 * q];
            const double dot = (nrm[0] * (co[0] - ci[0]) + nrm[1] * (co[1] - ci[1])) +
                               nrm[2] * (co[2] - ci[2]);
            if (dot < 0) std::swap(v1, v2);
            int32_t *T = &res->T[3 * (size_t)(toff[s] + q)];
            T[0] = (int32_t)v0;
            T[1] = (int32_t)v1;
            T[2] = (int32_t)v2;
        }
    }
    g_last = res;
    *nv_out = nv;
    *nt_out = ntri;
    return 0;
}

// Copies the last mg_march result (V [nv][3], T [nt][3]) and frees it.
int mg_march_fetch(double *V, int32_t *T) {
    if (!g_last) return -1;
    std::memcpy(V, g_last->V.data(), g_last->V.size() * sizeof(double));
    std::memcpy(T, g_last->T.data(), g_last->T.size() * sizeof(int32_t));
    delete g_last;
    g_last = nullptr;
    return 0;
}

}  // extern "C"
