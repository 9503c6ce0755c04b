// Host side of the XZZX SA decoder library: lattice geometry, noise model,
// energy weights, beta schedules, integer acceptance thresholds and the
// per-plan tables uploaded to the GPU (generator descriptors, move-energy
// lookup, threshold table, greedy-matching distance tables).
//
// Everything here runs once per plan (a lattice, a set of weights and a beta
// schedule); the per-syndrome work runs in xzzx_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <queue>
#include <tuple>

#include "xzzx_internal.h"

namespace xzzx {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

// ---------------------------------------------------------------------------
// Lattices (Sec. II).  Slot order of every generator: X_left, Z_up, Z_down,
// X_right with Pauli codes 2, 1, 1, 2 (Eq. (1)).
// ---------------------------------------------------------------------------
static const uint8_t kSlotPauli[4] = {2, 1, 1, 2};

namespace {
struct FaceRec {
    int sort_a, sort_b;   // row-major key (row, column)
    int q[4];
    int cls, colour;
    int cx, cy;
};
}  // namespace

static void finish_lattice(Lattice &L, std::vector<FaceRec> &faces)
{
    std::sort(faces.begin(), faces.end(), [](const FaceRec &a, const FaceRec &b) {
        return std::tie(a.sort_a, a.sort_b) < std::tie(b.sort_a, b.sort_b);
    });
    L.nstab = (int)faces.size();
    L.per_class = L.nstab / 4;
    L.fq.assign(4 * L.nstab, -1);
    L.fm.assign(4 * L.nstab, 0);
    L.fclass.resize(L.nstab);
    L.fcolour.resize(L.nstab);
    L.frank.resize(L.nstab);
    L.fcx.resize(L.nstab);
    L.fcy.resize(L.nstab);
    L.by_class.assign(4 * L.per_class, -1);
    for (int f = 0; f < L.nstab; ++f) {
        for (int s = 0; s < 4; ++s) {
            L.fq[4 * f + s] = faces[f].q[s];
            L.fm[4 * f + s] = faces[f].q[s] >= 0 ? kSlotPauli[s] : 0;
        }
        L.fclass[f] = faces[f].cls;
        L.fcolour[f] = faces[f].colour;
        L.fcx[f] = faces[f].cx;
        L.fcy[f] = faces[f].cy;
    }
    // Rank inside each colour class: face-id order on the rotated lattice;
    // on the planar lattice row-major over ((x + y)/2, (x - y)/2), the face's
    // 2 x 2 block in the frame turned by 45 degrees, so that consecutive ranks
    // share a row pair of the packed-row kernel.  The rank names the random
    // word each generator draws.
    for (int k = 0; k < 4; ++k) {
        std::vector<int> members;
        for (int f = 0; f < L.nstab; ++f)
            if (L.fclass[f] == k) members.push_back(f);
        if (L.layout == XZZX_PLANAR)
            std::sort(members.begin(), members.end(), [&](int a, int b) {
                return std::make_pair((L.fcx[a] + L.fcy[a]) / 2, (L.fcx[a] - L.fcy[a]) / 2) <
                       std::make_pair((L.fcx[b] + L.fcy[b]) / 2, (L.fcx[b] - L.fcy[b]) / 2);
            });
        for (int r = 0; r < (int)members.size(); ++r) {
            L.frank[members[r]] = r;
            if (r < L.per_class) L.by_class[k * L.per_class + r] = members[r];
        }
    }
}

int build_lattice(int layout, int d, Lattice &L)
{
    if (d < 3 || d > kMaxD || (d % 2) == 0) {
        set_error("lattice distance must be odd and in [3, 31]");
        return XZZX_EINVAL;
    }
    L = Lattice();
    L.layout = layout;
    L.d = d;
    std::vector<FaceRec> faces;
    if (layout == XZZX_ROTATED) {
        L.nq = d * d;
        auto qubit = [d](int x, int y) { return (x < 0 || y < 0 || x >= d || y >= d) ? -1 : y * d + x; };
        for (int j = -1; j < d; ++j) {
            for (int i = -1; i < d; ++i) {
                const bool col_in = (i >= 0 && i <= d - 2), row_in = (j >= 0 && j <= d - 2);
                bool gen;
                if (col_in && row_in) gen = true;                        // bulk
                else if (col_in && j == -1) gen = (i % 2) == 1;          // bottom edge
                else if (col_in && j == d - 1) gen = (i % 2) == 0;       // top edge
                else if (row_in && i == -1) gen = (j % 2) == 0;          // left edge
                else if (row_in && i == d - 1) gen = (j % 2) == 1;       // right edge
                else gen = false;                                        // corners
                if (!gen) continue;
                FaceRec r{};
                r.sort_a = j;
                r.sort_b = i;
                r.q[0] = qubit(i, j);
                r.q[1] = qubit(i + 1, j);
                r.q[2] = qubit(i, j + 1);
                r.q[3] = qubit(i + 1, j + 1);
                r.cls = ((i + 1) & 1) | (((j + 1) & 1) << 1);
                r.colour = ((i + j) % 2 + 2) % 2;
                r.cx = i;
                r.cy = j;
                faces.push_back(r);
            }
        }
        finish_lattice(L, faces);
        L.lx.assign(L.nq, 0);
        L.lz.assign(L.nq, 0);
        for (int t = 0; t < d; ++t) {
            L.lz[qubit(t, 0)] = (t % 2 == 0) ? 1 : 2;   // row y = 0, left to right
            L.lx[qubit(0, t)] = (t % 2 == 0) ? 2 : 1;   // column x = 0, bottom to top
        }
    } else if (layout == XZZX_PLANAR) {
        // Doubled coordinates; (odd, even) qubits first, then (even, odd).
        L.nq = d * d + (d - 1) * (d - 1);
        auto qubit = [d](int x, int y) -> int {
            if ((x & 1) && !(y & 1) && x >= 3 && x <= 2 * d - 1 && y >= 2 && y <= 2 * d - 2)
                return (y / 2 - 1) * (d - 1) + (x - 3) / 2;
            if (!(x & 1) && (y & 1) && x >= 2 && x <= 2 * d && y >= 1 && y <= 2 * d - 1)
                return (d - 1) * (d - 1) + (y / 2) * d + (x / 2 - 1);
            return -1;
        };
        auto add = [&](int x, int y, int colour) {
            FaceRec r{};
            r.sort_a = y;
            r.sort_b = x;
            r.q[0] = qubit(x - 1, y);
            r.q[1] = qubit(x, y + 1);
            r.q[2] = qubit(x, y - 1);
            r.q[3] = qubit(x + 1, y);
            auto fl = [](int a) { return (a >= 0) ? a / 2 : -((1 - a) / 2); };
            r.cls = (fl(x + y) & 1) | ((fl(x - y) & 1) << 1);
            r.colour = colour;
            r.cx = x;
            r.cy = y;
            faces.push_back(r);
        };
        for (int i = 1; i <= d; ++i)           // white faces (i, j) at (2i, 2j)
            for (int j = 1; j <= d - 1; ++j) add(2 * i, 2 * j, 0);
        for (int i = 1; i <= d - 1; ++i)       // gray faces (i, j) at (2i+1, 2j-1)
            for (int j = 1; j <= d; ++j) add(2 * i + 1, 2 * j - 1, 1);
        finish_lattice(L, faces);
        L.lx.assign(L.nq, 0);
        L.lz.assign(L.nq, 0);
        for (int t = 1; t <= d; ++t) {
            L.lz[qubit(2 * t, 1)] = 1;       // bottom row of (even, odd) qubits
            L.lx[qubit(2, 2 * t - 1)] = 2;   // left column of (even, odd) qubits
        }
    } else {
        set_error("unknown lattice layout");
        return XZZX_EINVAL;
    }
    for (int k = 0; k < 4; ++k)
        for (int m = 0; m < L.per_class; ++m)
            if (L.by_class[k * L.per_class + m] < 0) {
                set_error("colour classes are not of equal size");
                return XZZX_EINVAL;
            }
    // every kernel moves the generators of one class at once (or merges their
    // flips), which is exact only if a class's generators act on disjoint
    // qubits: checked for every lattice built
    std::vector<int> owner(L.nq, -1);
    for (int k = 0; k < 4; ++k) {
        for (int m = 0; m < L.per_class; ++m) {
            const int f = L.by_class[k * L.per_class + m];
            for (int s = 0; s < 4; ++s) {
                const int q = L.fq[4 * f + s];
                if (q < 0) continue;
                if (owner[q] == k) { set_error("a colour class has generators sharing a qubit"); return XZZX_EINVAL; }
                owner[q] = k;
            }
        }
    }
    return XZZX_OK;
}

// ---------------------------------------------------------------------------
// Acceptance threshold of Alg. 3 on a uint32 draw u (r = u / 2^32): a move
// with dE > 0 (units of 2^-16 nats) is accepted iff
// u < ceil(2^32 exp(-beta dE 2^-16)), threshold clamped to 2^32-1.
// ---------------------------------------------------------------------------
uint32_t accept_threshold(double beta, int64_t dE)
{
    if (dE <= 0) return 0xFFFFFFFFu;
    const double prob = std::exp(-(beta * static_cast<double>(dE)) * 0x1p-16);
    const double t = std::ceil(std::ldexp(prob, 32));
    return t >= 4294967295.0 ? 0xFFFFFFFFu : static_cast<uint32_t>(t);
}

// ---------------------------------------------------------------------------
// Plan tables.
// ---------------------------------------------------------------------------
// Ladder kernel: the tables as above with thresholds per level, 64 chains of
// nq / 16 + 1 packed words, and each lane's energy and level slot.
size_t Plan::lds_bytes_ladder() const
{
    size_t off = 0;
    off += sizeof(Desc) * 4 * lat.per_class;
    off += 256 * (size_t)ntypes;
    off = (off + 7) & ~size_t(7);
    off += 8 * dE.size() * (size_t)std::max(ladder_k, 1);
    off = (off + 15) & ~size_t(15);
    off += 4 * (size_t)(lat.nq / 16 + 1) * kWave;
    off += 8 * (size_t)kWave;
    return (off + 15) & ~size_t(15);
}

// Random-site kernel: the tables as above (descriptors in face-id order),
// then 64 chains of nq / 16 + 1 packed words.
size_t Plan::lds_bytes_site() const
{
    size_t off = 0;
    off += sizeof(Desc) * 4 * lat.per_class;
    off += 256 * (size_t)ntypes;
    off = (off + 7) & ~size_t(7);
    off += 8 * dE.size();
    off = (off + 15) & ~size_t(15);
    off += 4 * (size_t)(lat.nq / 16 + 1) * kWave;
    return (off + 15) & ~size_t(15);
}

size_t Plan::lds_bytes_anneal(int lanes_per_chain) const
{
    const int C = kWave / lanes_per_chain;
    size_t off = 0;
    off += sizeof(Desc) * 4 * lat.per_class;         // descriptors
    off += 256 * (size_t)ntypes;                     // move-energy ranks
    off = (off + 7) & ~size_t(7);
    off += 8 * dE.size();                            // (dE, threshold) pairs
    off = (off + 15) & ~size_t(15);
    off += (size_t)(lat.nq + 1) * C;                 // states, one scratch byte per chain
    return (off + 15) & ~size_t(15);
}

// Packed-row grid.  Rotated: rows y = -1..d and columns x = -1..d (padding
// around the d x d qubits).  Planar: the lattice turned by 45 degrees, where
// qubit (x, y) of the doubled coordinates sits at row (x + y - 1)/2 - 1 and
// column (x - y - 1)/2 + d - 1, and generator (x, y) covers the 2 x 2 block
// with top-left corner at row (x + y)/2 - 2, column (x - y)/2 + d - 2: X on
// the diagonal, Z on the anti-diagonal, as on the rotated lattice.  Its 2d - 1
// rows hold a diamond of qubits; columns 2d - 1 and 2d are padding.
static int rows_of(const Lattice &L) { return L.layout == XZZX_ROTATED ? L.d + 2 : 2 * L.d - 1; }
static int row_columns(const Lattice &L) { return L.layout == XZZX_ROTATED ? L.d + 2 : 2 * L.d + 1; }

size_t Plan::lds_bytes_rows() const
{
    size_t off = 256 * (size_t)ntypes;               // move-energy ranks
    off = (off + 7) & ~size_t(7);
    off += 8 * dE.size();                            // (dE, threshold) pairs
    off = (off + 15) & ~size_t(15);
    off += (size_t)4 * kWave * row_words * rows_of(lat);
    return (off + 15) & ~size_t(15);
}

template <int D>
static bool schedule_matches(const std::vector<uint32_t> &rowface, int mpad)
{
    constexpr RotSchedule<D> S{};
    if (S.MP != mpad) return false;
    for (int k = 0; k < 4; ++k)
        for (int m = 0; m < mpad; ++m) {
            const RotGen &g = S.g[k][m];
            if (rowface[k * mpad + m] != (g.Y | ((uint32_t)g.bo << 8) | ((uint32_t)g.shp << 16))) return false;
        }
    return true;
}

static bool static_schedule_matches(int d, const std::vector<uint32_t> &rowface, int mpad)
{
    switch (d) {
    case 3: return schedule_matches<3>(rowface, mpad);
    case 5: return schedule_matches<5>(rowface, mpad);
    case 7: return schedule_matches<7>(rowface, mpad);
    case 9: return schedule_matches<9>(rowface, mpad);
    case 11: return schedule_matches<11>(rowface, mpad);
    case 13: return schedule_matches<13>(rowface, mpad);
    case 15: return schedule_matches<15>(rowface, mpad);
    case 17: return schedule_matches<17>(rowface, mpad);
    case 19: return schedule_matches<19>(rowface, mpad);
    case 21: return schedule_matches<21>(rowface, mpad);
    case 23: return schedule_matches<23>(rowface, mpad);
    case 25: return schedule_matches<25>(rowface, mpad);
    case 27: return schedule_matches<27>(rowface, mpad);
    case 29: return schedule_matches<29>(rowface, mpad);
    case 31: return schedule_matches<31>(rowface, mpad);
    default: return false;
    }
}

// Packed-row layout (rotated lattice): the padded grid has columns and rows
// -1..d; a row of 2-bit codes takes 2(d+2) bits, so 1 word for d <= 13 and 2
// words for d <= 29.
// The default kernel: packed rows on rotated lattices, and on planar ones
// where the kernel specialised to d applies; otherwise the byte-state kernel
// on the planar lattice, which measured faster than the generic packed rows
// at d = 9 (two words per row, half the grid padding).  Every kernel stays
// available to set_kernel and the autotuner.
static bool rows_by_default(const Plan &P)
{
    return P.static_ok || P.planar_ok || (P.row_words && P.lat.layout == XZZX_ROTATED);
}

static int row_words_for(const Lattice &L)
{
    const int bits = 2 * row_columns(L);
    return bits <= 32 ? 1 : (bits <= 64 ? 2 : 0);
}

static int default_lanes(const Lattice &L)
{
    // Largest number of chains per wavefront whose interleaved states fit in
    // 16 KiB of LDS; the remaining lanes split the generators of one class.
    int C = kWave;
    while (C > 1 && (size_t)(L.nq + 1) * C > 16384) C /= 2;
    return kWave / C;
}

namespace {
struct Graph {
    int n = 0;
    std::vector<int32_t> col_face;           // node -> face
    std::vector<std::array<int32_t, 3>> adj;  // [n][4] (eid, other, w), eid -1 = none
    std::vector<int32_t> dint, db;
};
}  // namespace

static int build_graphs(const Lattice &L, const int32_t wg[2], Graph G[2])
{
    std::vector<int> node(L.nstab, -1);
    for (int g = 0; g < 2; ++g) {
        G[g] = Graph();
        for (int f = 0; f < L.nstab; ++f)
            if (L.fcolour[f] == g) { node[f] = G[g].n++; G[g].col_face.push_back(f); }
        G[g].adj.assign(4 * G[g].n, {-1, -1, 0});
    }
    // A slot with Pauli m on qubit q is flipped by the component of q that
    // anticommutes with m: the Z component (code 1) for m = X, the X component
    // (code 2) for m = Z.  Collect, per (qubit, component), the faces it flips.
    std::map<int, std::vector<int>> flips;  // edge id -> faces
    for (int f = 0; f < L.nstab; ++f)
        for (int s = 0; s < 4; ++s) {
            const int q = L.fq[4 * f + s];
            if (q < 0) continue;
            const int comp_is_x = (L.fm[4 * f + s] == 1) ? 1 : 0;
            flips[2 * q + comp_is_x].push_back(f);
        }
    for (auto &kv : flips) {
        const int eid = kv.first;
        const auto &fs = kv.second;
        if (fs.size() > 2 || L.fcolour[fs[0]] != L.fcolour[fs.back()]) {
            set_error("decoding graph is not a graph");
            return XZZX_EINVAL;
        }
        const int g = L.fcolour[fs[0]];
        const int32_t w = (eid & 1) ? wg[0] : wg[1];
        for (size_t h = 0; h < fs.size(); ++h) {
            const int u = node[fs[h]];
            const int other = fs.size() == 2 ? node[fs[1 - h]] : -1;
            int slot = 0;
            while (slot < 4 && G[g].adj[4 * u + slot][0] >= 0) ++slot;
            if (slot == 4) { set_error("node degree above 4"); return XZZX_EINVAL; }
            G[g].adj[4 * u + slot] = {eid, other, w};   // edge ids arrive in ascending order
        }
    }
    for (int g = 0; g < 2; ++g) {
        const int n = G[g].n;
        G[g].dint.assign((size_t)n * n, INT32_MAX);
        G[g].db.assign(n, INT32_MAX);
        using QE = std::pair<int64_t, int>;
        auto dijkstra = [&](std::vector<int64_t> &dist, std::priority_queue<QE, std::vector<QE>, std::greater<QE>> &pq) {
            while (!pq.empty()) {
                auto [dv, v] = pq.top();
                pq.pop();
                if (dv != dist[v]) continue;
                for (int s = 0; s < 4; ++s) {
                    const auto &e = G[g].adj[4 * v + s];
                    if (e[0] < 0 || e[1] < 0) continue;
                    const int64_t nd = dv + e[2];
                    if (nd < dist[e[1]]) { dist[e[1]] = nd; pq.push({nd, e[1]}); }
                }
            }
        };
        std::vector<int64_t> dist(n);
        for (int src = 0; src < n; ++src) {
            std::fill(dist.begin(), dist.end(), INT64_MAX);
            std::priority_queue<QE, std::vector<QE>, std::greater<QE>> pq;
            dist[src] = 0;
            pq.push({0, src});
            dijkstra(dist, pq);
            for (int v = 0; v < n; ++v) {
                if (dist[v] >= INT32_MAX) { set_error("decoding graph disconnected or too heavy"); return XZZX_ERANGE; }
                G[g].dint[(size_t)src * n + v] = (int32_t)dist[v];
            }
        }
        // distance to the boundary: shortest path to a virtual node joined by
        // every half-edge
        std::fill(dist.begin(), dist.end(), INT64_MAX);
        std::priority_queue<QE, std::vector<QE>, std::greater<QE>> pq;
        for (int v = 0; v < n; ++v)
            for (int s = 0; s < 4; ++s) {
                const auto &e = G[g].adj[4 * v + s];
                if (e[0] >= 0 && e[1] < 0 && e[2] < dist[v]) { dist[v] = e[2]; pq.push({e[2], v}); }
            }
        dijkstra(dist, pq);
        for (int v = 0; v < n; ++v) {
            if (dist[v] >= INT32_MAX) { set_error("no boundary reachable"); return XZZX_ERANGE; }
            G[g].db[v] = (int32_t)dist[v];
        }
    }
    return XZZX_OK;
}

static inline Desc pack_desc(const Lattice &L, int f, int shape)
{
    uint32_t q[4];
    for (int s = 0; s < 4; ++s) q[s] = L.fq[4 * f + s] >= 0 ? (uint32_t)L.fq[4 * f + s] : (uint32_t)L.nq;
    Desc d;
    d.x = q[0] | (q[1] << 16);
    d.y = q[2] | (q[3] << 16) | ((uint32_t)shape << 27);
    return d;
}

int build_plan(const Lattice &L, const int32_t w[4], const int32_t wg[2], const double *beta,
               int n_sweeps, Plan &P)
{
    if (n_sweeps < 0 || (n_sweeps > 0 && !beta)) { set_error("bad schedule"); return XZZX_EINVAL; }
    if (w[0] != 0 || w[1] <= 0 || w[2] <= 0 || w[3] <= 0 || wg[0] <= 0 || wg[1] <= 0) {
        set_error("weights must be positive (w[0] = 0)");
        return XZZX_EINVAL;
    }
    const int32_t wmax = std::max(w[1], std::max(w[2], w[3]));
    if ((int64_t)L.nq * wmax >= (int64_t)1 << 31) { set_error("energy would overflow int32"); return XZZX_ERANGE; }
    if (L.nq + 1 >= 2048) { set_error("lattice too large for 11-bit qubit indices"); return XZZX_ERANGE; }
    P.lat = L;
    std::memcpy(P.W, w, sizeof(P.W));
    std::memcpy(P.Wg, wg, sizeof(P.Wg));
    P.n_sweeps = n_sweeps;
    P.beta.assign(beta, beta + n_sweeps);
    for (double b : P.beta)
        if (!(b >= 0.0) || !std::isfinite(b)) { set_error("beta must be finite and >= 0"); return XZZX_EINVAL; }

    // shapes = which of the four slots exist, numbered in descending mask
    // order (the canonical numbering the specialised kernels assume)
    std::vector<int> shape_of_face(L.nstab), mask_of_face(L.nstab), shapes;
    for (int f = 0; f < L.nstab; ++f) {
        int mask = 0;
        for (int s = 0; s < 4; ++s) if (L.fq[4 * f + s] >= 0) mask |= 1 << s;
        mask_of_face[f] = mask;
        if (std::find(shapes.begin(), shapes.end(), mask) == shapes.end()) shapes.push_back(mask);
    }
    std::sort(shapes.begin(), shapes.end(), std::greater<int>());
    for (int f = 0; f < L.nstab; ++f)
        shape_of_face[f] = (int)(std::find(shapes.begin(), shapes.end(), mask_of_face[f]) - shapes.begin());
    // a null shape (no slot present, energy change 0) pads the packed-row
    // generator lists to whole Philox blocks
    const int null_shape = (int)shapes.size();
    shapes.push_back(0);
    P.ntypes = (int)shapes.size();
    // move energy of every (shape, slot pattern); absent slots contribute 0,
    // whatever their (scratch) byte holds
    std::vector<int32_t> lut_de(256 * P.ntypes);
    std::vector<int32_t> all;
    for (int t = 0; t < P.ntypes; ++t)
        for (int pat = 0; pat < 256; ++pat) {
            int32_t de = 0;
            for (int s = 0; s < 4; ++s) {
                if (!(shapes[t] >> s & 1)) continue;
                const int c = (pat >> (2 * s)) & 3;
                de += w[c ^ kSlotPauli[s]] - w[c];
            }
            lut_de[256 * t + pat] = de;
            all.push_back(de);
        }
    std::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    if ((int)all.size() > kMaxRanks) { set_error("too many distinct move energies"); return XZZX_ERANGE; }
    P.dE = all;
    P.kneg = (int)(std::upper_bound(all.begin(), all.end(), 0) - all.begin());
    std::vector<uint8_t> lut(256 * P.ntypes);
    for (size_t i = 0; i < lut.size(); ++i)
        lut[i] = (uint8_t)(std::lower_bound(all.begin(), all.end(), lut_de[i]) - all.begin());
    const int nranks = (int)all.size();
    std::vector<uint32_t> thr((size_t)std::max(n_sweeps, 1) * nranks, 0xFFFFFFFFu);
    for (int t = 0; t < n_sweeps; ++t)
        for (int r = 0; r < nranks; ++r) thr[(size_t)t * nranks + r] = accept_threshold(P.beta[t], all[r]);

    P.row_words = row_words_for(L);
    // packed-row descriptors by (class, rank), each class padded to a
    // multiple of 4 entries so a block of four is read at once
    const int mpad = 4 * ((L.per_class + 3) / 4);
    std::vector<uint32_t> rowface(4 * mpad, 0);
    std::vector<uint32_t> qpos(L.nq, 0);
    if (L.layout == XZZX_ROTATED) {
        for (int q = 0; q < L.nq; ++q) qpos[q] = (uint32_t)((q / L.d + 1) << 8) | (uint32_t)(q % L.d + 1);
    } else if (P.row_words) {
        // planar slots: 0 top-left (X), 1 bottom-left (Z), 2 top-right (Z),
        // 3 bottom-right (X) of the generator's block; the packed-row
        // pattern orders them top-left, top-right, bottom-left, bottom-right,
        // so a generator takes the shape with slots 1 and 2 exchanged
        auto swap12 = [](int m) { return (m & 9) | ((m & 2) << 1) | ((m & 4) >> 1); };
        std::vector<int> rows_shape(L.nstab, -1);
        for (int f = 0; f < L.nstab; ++f) {
            const int want = swap12(mask_of_face[f]);
            for (int t = 0; t < (int)shapes.size(); ++t)
                if (shapes[t] == want) rows_shape[f] = t;
            if (rows_shape[f] < 0) P.row_words = 0;   // exchanged shape absent: no packed-row kernel
        }
        std::vector<int> placed(L.nq, 0);
        const int d = L.d;
        for (int f = 0; f < L.nstab && P.row_words; ++f) {
            const int x = L.fcx[f], y = L.fcy[f];
            const int top = (x + y) / 2 - 2, left = (x - y) / 2 + d - 2;
            const int dy[4] = {0, 1, 0, 1}, dx[4] = {0, 0, 1, 1};
            for (int sl = 0; sl < 4; ++sl) {
                const int q = L.fq[4 * f + sl];
                if (q < 0) continue;
                const uint32_t p = (uint32_t)((top + dy[sl]) << 8) | (uint32_t)(left + dx[sl]);
                if (placed[q] && qpos[q] != p) { set_error("inconsistent planar row positions"); return XZZX_EINVAL; }
                placed[q] = 1;
                qpos[q] = p;
            }
        }
        for (int q = 0; q < L.nq && P.row_words; ++q)
            if (!placed[q]) { set_error("planar qubit outside every generator"); return XZZX_EINVAL; }
        if (P.row_words) {
            const uint32_t pad = 0u | ((2u * (uint32_t)(2 * d - 1)) << 8) | ((uint32_t)null_shape << 16);
            for (int k = 0; k < 4; ++k)
                for (int m = 0; m < mpad; ++m) {
                    if (m >= L.per_class) { rowface[k * mpad + m] = pad; continue; }
                    const int f = L.by_class[k * L.per_class + m];
                    const int x = L.fcx[f], y = L.fcy[f];
                    const uint32_t Y = (uint32_t)((x + y) / 2 - 2), C = (uint32_t)((x - y) / 2 + d - 2);
                    rowface[k * mpad + m] = Y | ((2u * C) << 8) | ((uint32_t)rows_shape[f] << 16);
                }
        }
    }
    if (L.layout == XZZX_ROTATED && L.d <= kStaticMaxD) {
        // padding entries: the null shape on the nibble at column d+1 of rows
        // 0 and 1, which holds only padding bits (never a qubit)
        const uint32_t pad = 0u | ((2u * (uint32_t)(L.d + 1)) << 8) | ((uint32_t)null_shape << 16);
        for (int k = 0; k < 4; ++k)
            for (int m = 0; m < mpad; ++m) {
                if (m >= L.per_class) { rowface[k * mpad + m] = pad; continue; }
                const int f = L.by_class[k * L.per_class + m];
                const uint32_t Y = (uint32_t)(L.fcy[f] + 1), X = (uint32_t)(L.fcx[f] + 1);
                rowface[k * mpad + m] = Y | ((2u * X) << 8) | ((uint32_t)shape_of_face[f] << 16);
            }
    }
    // the planar kernel specialised to d applies when its compile-time
    // schedule and qubit positions are exactly this plan's tables
    P.planar_ok = 0;
    if (L.layout == XZZX_PLANAR && P.row_words && L.d <= kPlanarStaticMaxD && nranks <= kStaticRanks &&
        shapes == std::vector<int>(kPlanarShapeMasks, kPlanarShapeMasks + 6) &&
        planar_schedule_matches(L.d, rowface, mpad, qpos))
        P.planar_ok = 1;
    P.planar_d = P.planar_ok ? L.d : 0;
    // the specialised packed-row kernel applies when its compile-time
    // schedule is exactly this plan's table
    P.static_d = 0;
    if (L.layout == XZZX_ROTATED && L.d >= kStaticMinD && L.d <= kStaticMaxD &&
        nranks <= kStaticRanks && static_schedule_matches(L.d, rowface, mpad))
        P.static_d = L.d;
    P.static_ok = P.static_d ? 1 : 0;
    // its rows hold the d qubits and one spare column: 2(d + 1) bits
    P.static_words = P.static_ok ? (2 * (L.d + 1) + 31) / 32 : 0;
    std::vector<Desc> desc(4 * L.per_class), fdesc(L.nstab);
    for (int f = 0; f < L.nstab; ++f) fdesc[f] = pack_desc(L, f, shape_of_face[f]);
    for (int k = 0; k < 4; ++k)
        for (int m = 0; m < L.per_class; ++m) desc[k * L.per_class + m] = fdesc[L.by_class[k * L.per_class + m]];

    Graph G[2];
    int rc = build_graphs(L, wg, G);
    if (rc) return rc;

    // one device allocation: [PlanDev][tables...], 256-byte aligned pieces
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = (off + bytes + 255) & ~size_t(255); return o; };
    const size_t o_hdr = take(sizeof(PlanDev));
    const size_t o_rowface = take(rowface.size() * 4);
    const size_t o_desc = take(desc.size() * sizeof(Desc));
    const size_t o_fdesc = take(fdesc.size() * sizeof(Desc));
    const size_t o_lut = take(lut.size());
    const size_t o_de = take(all.size() * 4);
    const size_t o_thr = take(thr.size() * 4);
    const size_t o_lx = take(L.nq);
    const size_t o_lz = take(L.nq);
    const size_t o_qpos = take(qpos.size() * 4);
    size_t o_cf[2], o_dint[2], o_db[2], o_adj[2];
    for (int g = 0; g < 2; ++g) {
        o_cf[g] = take(G[g].n * 4);
        o_dint[g] = take((size_t)G[g].n * G[g].n * 4);
        o_db[g] = take(G[g].n * 4);
        o_adj[g] = take((size_t)G[g].n * 4 * sizeof(int4));
    }
    P.dbytes = off;
    if (hipGetDevice(&P.device) != hipSuccess) { set_error("hipGetDevice failed"); return XZZX_EDEVICE; }
    if (hipMalloc(&P.dmem, P.dbytes) != hipSuccess) { P.dmem = nullptr; set_error("hipMalloc of plan tables failed"); return XZZX_ENOMEM; }
    std::vector<uint8_t> host(P.dbytes, 0);
    auto put = [&](size_t o, const void *src, size_t n) { if (n) std::memcpy(host.data() + o, src, n); };
    put(o_rowface, rowface.data(), rowface.size() * 4);
    put(o_desc, desc.data(), desc.size() * sizeof(Desc));
    put(o_fdesc, fdesc.data(), fdesc.size() * sizeof(Desc));
    put(o_lut, lut.data(), lut.size());
    put(o_de, all.data(), all.size() * 4);
    put(o_thr, thr.data(), thr.size() * 4);
    put(o_lx, L.lx.data(), L.nq);
    put(o_lz, L.lz.data(), L.nq);
    put(o_qpos, qpos.data(), qpos.size() * 4);
    for (int g = 0; g < 2; ++g) {
        put(o_cf[g], G[g].col_face.data(), G[g].n * 4);
        put(o_dint[g], G[g].dint.data(), (size_t)G[g].n * G[g].n * 4);
        put(o_db[g], G[g].db.data(), G[g].n * 4);
        std::vector<int4> adj(G[g].n * 4);
        for (size_t i = 0; i < adj.size(); ++i) adj[i] = make_int4(G[g].adj[i][0], G[g].adj[i][1], G[g].adj[i][2], 0);
        put(o_adj[g], adj.data(), adj.size() * sizeof(int4));
    }
    auto *base = static_cast<uint8_t *>(P.dmem);
    PlanDev &h = P.hdev;
    h = PlanDev{};
    h.nq = L.nq;
    h.nstab = L.nstab;
    h.M = L.per_class;
    h.nblk = (L.per_class + 3) / 4;
    h.ntypes = P.ntypes;
    h.nranks = nranks;
    h.kneg = P.kneg;
    h.n_sweeps = n_sweeps;
    P.lanes_default = default_lanes(L);
    P.lanes = P.lanes_default;
    h.lanes = P.lanes;
    h.layout = L.layout;
    h.d = L.d;
    h.row_words = P.row_words;
    h.rows = rows_of(L);
    h.static_words = P.static_words;
    P.use_rows = rows_by_default(P) ? 1 : 0;
    h.rowface = reinterpret_cast<const uint32_t *>(base + o_rowface);
    std::memcpy(h.W, w, sizeof(h.W));
    h.desc = reinterpret_cast<const Desc *>(base + o_desc);
    h.face_desc = reinterpret_cast<const Desc *>(base + o_fdesc);
    h.lut = base + o_lut;
    h.dE = reinterpret_cast<const int32_t *>(base + o_de);
    h.thr = reinterpret_cast<const uint32_t *>(base + o_thr);
    h.lx = base + o_lx;
    h.lz = base + o_lz;
    h.qpos = reinterpret_cast<const uint32_t *>(base + o_qpos);
    for (int g = 0; g < 2; ++g) {
        h.ncol[g] = G[g].n;
        h.col_face[g] = reinterpret_cast<const int32_t *>(base + o_cf[g]);
        h.dint[g] = reinterpret_cast<const int32_t *>(base + o_dint[g]);
        h.db[g] = reinterpret_cast<const int32_t *>(base + o_db[g]);
        h.adj[g] = reinterpret_cast<const int4 *>(base + o_adj[g]);
    }
    put(o_hdr, &h, sizeof(PlanDev));
    P.ddev = reinterpret_cast<PlanDev *>(base + o_hdr);
    if (hipMemcpy(P.dmem, host.data(), P.dbytes, hipMemcpyHostToDevice) != hipSuccess) {
        set_error("upload of plan tables failed");
        return XZZX_EDEVICE;
    }
    return XZZX_OK;
}

}  // namespace xzzx

using namespace xzzx;

// ---------------------------------------------------------------------------
// C ABI: host-side calls.
// ---------------------------------------------------------------------------
extern "C" {

const char *xzzx_last_error(void) { return g_last_error.c_str(); }

int xzzx_version(void) { return 1; }

int xzzx_lattice_create(int layout, int d, xzzx_lattice **out)
{
    if (!out) { set_error("out is NULL"); return XZZX_EINVAL; }
    *out = nullptr;
    try {
        auto *h = new xzzx_lattice();
        int rc = build_lattice(layout, d, h->L);
        if (rc) { delete h; return rc; }
        *out = h;
        return XZZX_OK;
    } catch (...) {
        set_error("out of host memory");
        return XZZX_ENOMEM;
    }
}

void xzzx_lattice_destroy(xzzx_lattice *lat) { delete lat; }

int xzzx_lattice_info(const xzzx_lattice *lat, int *n_qubits, int *n_stabs, int *per_class)
{
    if (!lat) { set_error("lattice is NULL"); return XZZX_EINVAL; }
    if (n_qubits) *n_qubits = lat->L.nq;
    if (n_stabs) *n_stabs = lat->L.nstab;
    if (per_class) *per_class = lat->L.per_class;
    return XZZX_OK;
}

int xzzx_lattice_tables(const xzzx_lattice *lat, int32_t *face_qubits, uint8_t *face_paulis,
                        int32_t *face_class, int32_t *face_colour, int32_t *face_rank)
{
    if (!lat) { set_error("lattice is NULL"); return XZZX_EINVAL; }
    const Lattice &L = lat->L;
    if (face_qubits) std::memcpy(face_qubits, L.fq.data(), L.fq.size() * 4);
    if (face_paulis) std::memcpy(face_paulis, L.fm.data(), L.fm.size());
    if (face_class) std::memcpy(face_class, L.fclass.data(), L.nstab * 4);
    if (face_colour) std::memcpy(face_colour, L.fcolour.data(), L.nstab * 4);
    if (face_rank) std::memcpy(face_rank, L.frank.data(), L.nstab * 4);
    return XZZX_OK;
}

int xzzx_lattice_logicals(const xzzx_lattice *lat, uint8_t *lx, uint8_t *lz)
{
    if (!lat) { set_error("lattice is NULL"); return XZZX_EINVAL; }
    if (lx) std::memcpy(lx, lat->L.lx.data(), lat->L.nq);
    if (lz) std::memcpy(lz, lat->L.lz.data(), lat->L.nq);
    return XZZX_OK;
}

int xzzx_noise(double p, double eta, int convention, double pxyz[3])
{
    if (!pxyz || !(p > 0.0 && p < 0.5) || !(eta > 0.0) || !std::isfinite(eta)) {
        set_error("need 0 < p < 1/2 and finite eta > 0");
        return XZZX_EINVAL;
    }
    double px, py;
    if (convention == XZZX_BIAS_RATIO) {
        px = p / (2.0 * (eta + 1.0));
        py = p * eta / (eta + 1.0);
    } else if (convention == XZZX_BIAS_PAPER) {
        px = p / (eta + 2.0);
        py = p * eta / (eta + 2.0);
    } else {
        set_error("unknown bias convention");
        return XZZX_EINVAL;
    }
    pxyz[0] = px;
    pxyz[1] = py;
    pxyz[2] = px;
    return XZZX_OK;
}

int xzzx_weights(double p, const double pxyz[3], int32_t w[4], int32_t wg[2])
{
    if (!pxyz || !w || !wg || !(p > 0.0 && p < 0.5)) { set_error("need 0 < p < 1/2"); return XZZX_EINVAL; }
    const double keep = 1.0 - p;
    for (int i = 0; i < 3; ++i)
        if (!(pxyz[i] > 0.0 && pxyz[i] < keep)) { set_error("need 0 < p_P < 1-p"); return XZZX_EINVAL; }
    auto q16 = [](double ratio) { return (int32_t)std::llround(65536.0 * -std::log(ratio)); };
    w[0] = 0;
    w[1] = q16(pxyz[2] / keep);
    w[2] = q16(pxyz[0] / keep);
    w[3] = q16(pxyz[1] / keep);
    wg[0] = q16((pxyz[0] + pxyz[1]) / keep);
    wg[1] = q16((pxyz[2] + pxyz[1]) / keep);
    return XZZX_OK;
}

int xzzx_schedule(int kind, double b0, double b1, int n, double *beta)
{
    if (n < 0 || (n > 0 && !beta) || !(b0 >= 0.0) || !(b1 >= 0.0)) { set_error("bad schedule arguments"); return XZZX_EINVAL; }
    if ((kind == XZZX_SCHED_GEOMETRIC || kind == XZZX_SCHED_PAPER_LOG) && !(b0 > 0.0)) {
        set_error("schedule needs b0 > 0");
        return XZZX_EINVAL;
    }
    if (kind != XZZX_SCHED_LINEAR && kind != XZZX_SCHED_GEOMETRIC && kind != XZZX_SCHED_PAPER_LOG) {
        set_error("unknown schedule kind");
        return XZZX_EINVAL;
    }
    const double gamma = (kind == XZZX_SCHED_PAPER_LOG && n >= 2) ? (b1 / b0 - 1.0) / std::log((double)n) : 0.0;
    for (int t = 0; t < n; ++t) {
        const double frac = (n == 1) ? 0.0 : (double)t / (double)(n - 1);
        switch (kind) {
        case XZZX_SCHED_LINEAR: beta[t] = (n == 1) ? b0 : b0 + (b1 - b0) * frac; break;
        case XZZX_SCHED_GEOMETRIC: beta[t] = (n == 1) ? b0 : b0 * std::pow(b1 / b0, frac); break;
        default: beta[t] = b0 * (1.0 + gamma * std::log((double)(t + 1))); break;
        }
    }
    return XZZX_OK;
}

int xzzx_class_host(const xzzx_lattice *lat, const uint8_t *a, const uint8_t *b, int *cls)
{
    if (!lat || !a || !b || !cls) { set_error("NULL argument"); return XZZX_EINVAL; }
    const Lattice &L = lat->L;
    auto anti = [](int p, int q) { return (((p >> 1) & q) ^ (p & (q >> 1))) & 1; };
    for (int f = 0; f < L.nstab; ++f) {
        int s = 0;
        for (int k = 0; k < 4; ++k) {
            const int q = L.fq[4 * f + k];
            if (q >= 0) s ^= anti((a[q] ^ b[q]) & 3, L.fm[4 * f + k]);
        }
        if (s) { *cls = -1; return XZZX_OK; }
    }
    int vz = 0, vx = 0;
    for (int q = 0; q < L.nq; ++q) {
        const int e = (a[q] ^ b[q]) & 3;
        vz ^= anti(e, L.lz[q]);
        vx ^= anti(e, L.lx[q]);
    }
    static const int tab[2][2] = {{0, 3}, {1, 2}};   // [anticommutes with L_Z][with L_X]
    *cls = tab[vz][vx];
    return XZZX_OK;
}

int xzzx_plan_create(const xzzx_lattice *lat, const int32_t w[4], const int32_t wg[2],
                     const double *beta, int n_sweeps, xzzx_plan **out)
{
    if (!lat || !w || !wg || !out) { set_error("NULL argument"); return XZZX_EINVAL; }
    *out = nullptr;
    xzzx_plan *h = nullptr;
    try {
        h = new xzzx_plan();
    } catch (...) {
        set_error("out of host memory");
        return XZZX_ENOMEM;
    }
    int rc = build_plan(lat->L, w, wg, beta, n_sweeps, h->P);
    if (rc) {
        if (h->P.dmem) (void)hipFree(h->P.dmem);
        delete h;
        return rc;
    }
    *out = h;
    return XZZX_OK;
}

void xzzx_plan_destroy(xzzx_plan *plan)
{
    if (!plan) return;
    if (plan->P.dmem || plan->P.ladder_mem) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(plan->P.device);
        if (plan->P.dmem) (void)hipFree(plan->P.dmem);
        if (plan->P.ladder_mem) (void)hipFree(plan->P.ladder_mem);
        (void)hipSetDevice(cur);
    }
    delete plan;
}

int xzzx_plan_set_ladder(xzzx_plan *plan, int levels, double beta_lo, double beta_hi)
{
    if (!plan) { set_error("plan is NULL"); return XZZX_EINVAL; }
    Plan &P = plan->P;
    if (levels != 0 && levels != 1 && levels != 2 && levels != 4 && levels != 8 && levels != 16) {
        set_error("ladder levels must be 0 (off) or 1, 2, 4, 8, 16");
        return XZZX_EINVAL;
    }
    if (levels && P.order != XZZX_ORDER_COLOUR) { set_error("ladders run colour-class sweeps only"); return XZZX_EINVAL; }
    if (levels && (!(beta_lo >= 0.0) || !(beta_hi >= beta_lo) || !std::isfinite(beta_hi))) {
        set_error("ladder needs 0 <= beta_lo <= beta_hi, finite");
        return XZZX_EINVAL;
    }
    const int old_k = P.ladder_k;
    P.ladder_k = levels;
    if (levels && P.lds_bytes_ladder() > 65536) {
        P.ladder_k = old_k;
        set_error("ladder tables and chains do not fit in LDS");
        return XZZX_ERANGE;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != P.device) { P.ladder_k = old_k; set_error("plan was created on another device"); return XZZX_EINVAL; }
    void *mem = nullptr;
    if (levels) {
        // levels beta_k = beta_lo + k delta, and the exchange rule's powers
        const int nranks = P.nranks();
        const double delta = levels > 1 ? (beta_hi - beta_lo) / (double)(levels - 1) : 0.0;
        std::vector<uint32_t> thr((size_t)levels * nranks);
        for (int k = 0; k < levels; ++k) {
            const double b = levels > 1 ? beta_lo + (double)k * delta : beta_lo;
            for (int r = 0; r < nranks; ++r) thr[(size_t)k * nranks + r] = accept_threshold(b, P.dE[r]);
        }
        uint64_t R[32];
        const double r0 = std::ldexp(std::exp(-delta * 0x1p-16), 64);
        R[0] = r0 >= 18446744073709551615.0 ? UINT64_MAX : (uint64_t)r0;
        for (int i = 1; i < 32; ++i) R[i] = (uint64_t)(((unsigned __int128)R[i - 1] * R[i - 1]) >> 64);
        const size_t bytes = 256 + thr.size() * 4;
        if (hipMalloc(&mem, bytes) != hipSuccess) { P.ladder_k = old_k; set_error("hipMalloc of ladder tables failed"); return XZZX_ENOMEM; }
        std::vector<uint8_t> host(bytes, 0);
        std::memcpy(host.data(), R, sizeof(R));
        std::memcpy(host.data() + 256, thr.data(), thr.size() * 4);
        if (hipMemcpy(mem, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(mem);
            P.ladder_k = old_k;
            set_error("upload of ladder tables failed");
            return XZZX_EDEVICE;
        }
    }
    // publish the new tables in the device copy of the plan, then free the old ones
    PlanDev &h = P.hdev;
    h.ladder_k = levels;
    h.ladder_pow = levels ? static_cast<const uint64_t *>(mem) : nullptr;
    h.ladder_thr = levels ? reinterpret_cast<const uint32_t *>(static_cast<uint8_t *>(mem) + 256) : nullptr;
    if (hipMemcpy(P.ddev, &h, sizeof(PlanDev), hipMemcpyHostToDevice) != hipSuccess) {
        if (mem) (void)hipFree(mem);
        P.ladder_k = old_k;
        set_error("plan update failed");
        return XZZX_EDEVICE;
    }
    if (P.ladder_mem) (void)hipFree(P.ladder_mem);
    P.ladder_mem = mem;
    P.ladder_lo = beta_lo;
    P.ladder_hi = beta_hi;
    return XZZX_OK;
}

int xzzx_plan_set_kernel(xzzx_plan *plan, int kernel)
{
    if (!plan) { set_error("plan is NULL"); return XZZX_EINVAL; }
    if (kernel == XZZX_KERNEL_AUTO) {
        plan->P.use_rows = rows_by_default(plan->P) ? 1 : 0;
        plan->P.static_d = plan->P.static_ok ? plan->P.lat.d : 0;
        plan->P.planar_d = plan->P.planar_ok ? plan->P.lat.d : 0;
    } else if (kernel == XZZX_KERNEL_ROWS) {
        if (!plan->P.row_words && !plan->P.static_ok) {
            set_error("the packed-row kernel needs a rotated lattice with d <= 31 or a planar one with d <= 15");
            return XZZX_EINVAL;
        }
        plan->P.use_rows = 1;
        plan->P.static_d = plan->P.static_ok ? plan->P.lat.d : 0;
        plan->P.planar_d = plan->P.planar_ok ? plan->P.lat.d : 0;
    } else if (kernel == XZZX_KERNEL_ROWS_GENERIC) {
        if (!plan->P.row_words) { set_error("the generic packed-row kernel needs a rotated lattice with d <= 29 or a planar one with d <= 15"); return XZZX_EINVAL; }
        plan->P.use_rows = 1;
        plan->P.static_d = 0;
        plan->P.planar_d = 0;
    } else if (kernel == XZZX_KERNEL_BYTES) {
        plan->P.use_rows = 0;
    } else {
        set_error("unknown kernel");
        return XZZX_EINVAL;
    }
    return XZZX_OK;
}

int xzzx_plan_info(const xzzx_plan *plan, int *n_qubits, int *n_stabs, int *n_sweeps, int *n_dE,
                   int *lanes_per_chain, int *kernel)
{
    if (plan && kernel)
        *kernel = plan->P.order ? XZZX_KERNEL_SITE
                  : plan->P.ladder_k ? XZZX_KERNEL_LADDER
                  : !plan->P.use_rows ? XZZX_KERNEL_BYTES
                  : (plan->P.static_d || plan->P.planar_d) ? XZZX_KERNEL_ROWS : XZZX_KERNEL_ROWS_GENERIC;
    if (!plan) { set_error("plan is NULL"); return XZZX_EINVAL; }
    if (n_qubits) *n_qubits = plan->P.lat.nq;
    if (n_stabs) *n_stabs = plan->P.lat.nstab;
    if (n_sweeps) *n_sweeps = plan->P.n_sweeps;
    if (n_dE) *n_dE = (int)plan->P.dE.size();
    if (lanes_per_chain) *lanes_per_chain = plan->P.lanes;
    return XZZX_OK;
}

int xzzx_plan_set_order(xzzx_plan *plan, int order)
{
    if (!plan) { set_error("plan is NULL"); return XZZX_EINVAL; }
    if (order != XZZX_ORDER_COLOUR && order != XZZX_ORDER_RANDOM_SITE) { set_error("unknown step order"); return XZZX_EINVAL; }
    if (order != XZZX_ORDER_COLOUR && plan->P.ladder_k) { set_error("ladders run colour-class sweeps only"); return XZZX_EINVAL; }
    if (order == XZZX_ORDER_RANDOM_SITE) {
        if ((int64_t)plan->P.n_sweeps * plan->P.lat.nstab >= ((int64_t)1 << 31)) {
            set_error("random-site steps of a chain must number below 2^31");
            return XZZX_ERANGE;
        }
        if (plan->P.lds_bytes_site() > 65536) { set_error("random-site chains do not fit in LDS"); return XZZX_ERANGE; }
    }
    plan->P.order = order;
    return XZZX_OK;
}

int xzzx_plan_set_lanes(xzzx_plan *plan, int lanes_per_chain)
{
    if (!plan) { set_error("plan is NULL"); return XZZX_EINVAL; }
    int g = lanes_per_chain == 0 ? plan->P.lanes_default : lanes_per_chain;
    if (g < 1 || g > kWave || (g & (g - 1))) { set_error("lanes per chain must be a power of two in [1, 64]"); return XZZX_EINVAL; }
    if (plan->P.lds_bytes_anneal(g) > 65536) { set_error("chains per wavefront do not fit in LDS"); return XZZX_ERANGE; }
    plan->P.lanes = g;
    plan->P.hdev.lanes = g;
    plan->P.use_rows = (lanes_per_chain == 0 && rows_by_default(plan->P)) ? 1 : 0;
    if (hipMemcpy(&plan->P.ddev->lanes, &g, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
        set_error("plan update failed");
        return XZZX_EDEVICE;
    }
    return XZZX_OK;
}

}  // extern "C"
