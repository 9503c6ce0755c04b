// Internal data structures shared by the host plan builder (xzzx_host.cpp) and
// the gfx950 kernels (xzzx_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <functional>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/xzzx_sa.h"

namespace xzzx {

constexpr int kWave = 64;
constexpr int kMaxD = 31;
constexpr int kMaxGroups = 16;   // syndrome groups per persistent launch
constexpr int kMaxRanks = 255;   // distinct move energies per plan (u8 rank)
constexpr int kMaxTypes = 16;    // generator shapes (subset of the four slots)

// Generator descriptor, 8 bytes: the four slot qubits (X_left, Z_up, Z_down,
// X_right), an absent slot pointing at the per-chain scratch byte n_q, and the
// shape index used by the move-energy lookup.
//   x = q0 | q1 << 16,  y = q2 | (q3 << 16) | (shape << 27)
struct Desc {
    uint32_t x, y;
};

// Canonical generator shapes (slot-presence masks, slot s = bit s) in
// descending mask order; the plan numbers the shapes of a lattice in this
// order and appends the null shape (no slot) last.  On the rotated lattice
// these are: 15 bulk, 12 bottom edge, 10 left edge, 5 right edge, 3 top edge.
constexpr int kRotShapeMasks[6] = {15, 12, 10, 5, 3, 0};

// Compile-time generator schedule of the rotated lattice at distance D for
// the packed-row kernel specialised to D: for colour class k and rank m, the
// row Y = j + 1 of cell (i, j) and the bit offset 2(i + 1) of its nibble in
// the padded grid of the generic packed-row kernel (rows and columns -1..D),
// and its canonical shape.  This is the plan's own table, against which the
// host checks it.  Ranks run row-major over (j, i), as in the plan; each
// class is padded to a multiple of four with null generators on the padding
// nibble of rows 0 and 1.
struct RotGen {
    uint8_t Y, bo, shp;
};

template <int D>
struct RotSchedule {
    static constexpr int M = (D * D - 1) / 4;
    static constexpr int MP = (M + 3) / 4 * 4;
    RotGen g[4][MP];
    constexpr RotSchedule() : g{}
    {
        int cnt[4] = {0, 0, 0, 0};
        for (int j = -1; j < D; ++j)
            for (int i = -1; i < D; ++i) {
                const bool col_in = i >= 0 && i <= D - 2, row_in = j >= 0 && j <= D - 2;
                bool gen = false;
                if (col_in && row_in) gen = true;
                else if (col_in && j == -1) gen = (i % 2) == 1;
                else if (col_in && j == D - 1) gen = (i % 2) == 0;
                else if (row_in && i == -1) gen = (j % 2) == 0;
                else if (row_in && i == D - 1) gen = (j % 2) == 1;
                if (!gen) continue;
                int mask = 0;
                if (i >= 0 && j >= 0) mask |= 1;                  // X on (i, j)
                if (i <= D - 2 && j >= 0) mask |= 2;              // Z on (i+1, j)
                if (i >= 0 && j <= D - 2) mask |= 4;              // Z on (i, j+1)
                if (i <= D - 2 && j <= D - 2) mask |= 8;          // X on (i+1, j+1)
                int shp = 0;
                while (kRotShapeMasks[shp] != mask) ++shp;
                const int k = ((i + 1) & 1) | (((j + 1) & 1) << 1);
                g[k][cnt[k]++] = RotGen{(uint8_t)(j + 1), (uint8_t)(2 * (i + 1)), (uint8_t)shp};
            }
        for (int k = 0; k < 4; ++k)
            for (int m = cnt[k]; m < MP; ++m) g[k][m] = RotGen{0, (uint8_t)(2 * (D + 1)), 5};
    }
};

// Compile-time schedule of the planar lattice at distance D for the
// packed-row kernel specialised to it.  Turned by 45 degrees, qubit (x, y) of
// the doubled coordinates sits at row (x + y - 1)/2 - 1, column
// (x - y - 1)/2 + D - 1, and generator (x, y) covers the 2 x 2 block at row
// (x + y)/2 - 2, column (x - y)/2 + D - 2 (X on the diagonal, Z on the
// anti-diagonal); its slots 1 and 2 trade places in the block, so its shape
// is the one with those slots exchanged.  Ranks within a class run row-major
// over ((x + y)/2, (x - y)/2), as in the plan; each class is padded to a
// multiple of four with null generators on the padding columns 2D - 1, 2D of
// rows 0 and 1.  The qubit numbering is the plan's: (odd, even) qubits first,
// then (even, odd).  This is the plan's own table, against which the host
// checks it.
constexpr int kPlanarShapeMasks[6] = {15, 14, 13, 11, 7, 0};

template <int D>
struct PlanarSchedule {
    static constexpr int NS = 2 * D * (D - 1);
    static constexpr int M = NS / 4;
    static constexpr int MP = (M + 3) / 4 * 4;
    static constexpr int NQ = D * D + (D - 1) * (D - 1);
    RotGen g[4][MP];
    uint16_t qpos[NQ];   // row << 8 | column
    static constexpr int qubit(int x, int y)
    {
        if ((x & 1) && !(y & 1) && x >= 3 && x <= 2 * D - 1 && y >= 2 && y <= 2 * D - 2)
            return (y / 2 - 1) * (D - 1) + (x - 3) / 2;
        if (!(x & 1) && (y & 1) && x >= 2 && x <= 2 * D && y >= 1 && y <= 2 * D - 1)
            return (D - 1) * (D - 1) + (y / 2) * D + (x / 2 - 1);
        return -1;
    }
    constexpr PlanarSchedule() : g{}, qpos{}
    {
        int fx[NS] = {}, fy[NS] = {}, fk[NS] = {}, used[NS] = {};
        int n = 0;
        for (int i = 1; i <= D; ++i)
            for (int j = 1; j <= D - 1; ++j) { fx[n] = 2 * i; fy[n] = 2 * j; ++n; }
        for (int i = 1; i <= D - 1; ++i)
            for (int j = 1; j <= D; ++j) { fx[n] = 2 * i + 1; fy[n] = 2 * j - 1; ++n; }
        for (int f = 0; f < NS; ++f) {
            const int a = fx[f] + fy[f], b = fx[f] - fy[f];
            fk[f] = ((a / 2) & 1) | (((b >= 0 ? b / 2 : -((-b) / 2)) & 1) << 1);
        }
        for (int k = 0; k < 4; ++k) {
            int m = 0;
            for (;; ++m) {
                int best = -1;
                for (int f = 0; f < NS; ++f) {
                    if (used[f] || fk[f] != k) continue;
                    if (best < 0 || (fx[f] + fy[f] < fx[best] + fy[best]) ||
                        (fx[f] + fy[f] == fx[best] + fy[best] && fx[f] - fy[f] < fx[best] - fy[best]))
                        best = f;
                }
                if (best < 0) break;
                used[best] = 1;
                const int x = fx[best], y = fy[best];
                const int q[4] = {qubit(x - 1, y), qubit(x, y + 1), qubit(x, y - 1), qubit(x + 1, y)};
                int mask = 0;
                for (int sl = 0; sl < 4; ++sl) mask |= (q[sl] >= 0 ? 1 : 0) << sl;
                const int rows_mask = (mask & 9) | ((mask & 2) << 1) | ((mask & 4) >> 1);
                int shp = 0;
                while (kPlanarShapeMasks[shp] != rows_mask) ++shp;
                const int top = (x + y) / 2 - 2, left = (x - y) / 2 + D - 2;
                g[k][m] = RotGen{(uint8_t)top, (uint8_t)(2 * left), (uint8_t)shp};
                const int dy[4] = {0, 1, 0, 1}, dx[4] = {0, 0, 1, 1};
                for (int sl = 0; sl < 4; ++sl)
                    if (q[sl] >= 0) qpos[q[sl]] = (uint16_t)(((top + dy[sl]) << 8) | (left + dx[sl]));
            }
            for (; m < MP; ++m) g[k][m] = RotGen{0, (uint8_t)(2 * (2 * D - 1)), 5};
        }
    }
};
template <int D>
inline constexpr PlanarSchedule<D> kPlanarSchedule{};

// Planar distances with a specialised packed-row kernel (rows of 2D + 1
// columns in at most two words), and the host check that a plan's packed-row
// tables are its compile-time schedule.
constexpr int kPlanarStaticMaxD = 15;
bool planar_schedule_matches(int d, const std::vector<uint32_t> &rowface, int mpad, const std::vector<uint32_t> &qpos);

// Distances with a specialised packed-row kernel, and the largest number of
// distinct move energies its static tables hold.
constexpr int kStaticMinD = 3, kStaticMaxD = 31;
constexpr int kStaticRanks = 128;
// static LDS of a specialised kernel's workgroup: the u16 (shape, pattern)
// lookup of six shapes and the 16-byte move-energy entries
constexpr size_t kStaticLdsBytes = 2 * 256 * 6 + 16 * kStaticRanks;
// Rotated distances whose replica-exchange ladders run on a packed-row
// kernel specialised to d (every distance with such an annealing kernel).
constexpr int kLadderRowsMaxD = 31;
// The specialised kernel's state checkpoints (the replay of a syndrome's
// best chain starts from the last one before its E_min phase): every
// kCheckpointEvery sweeps, or sparser so that a chain keeps at most
// kMaxCheckpoints of them.
constexpr int kCheckpointEvery = 64;
constexpr int kMaxCheckpoints = 32;
// sweeps between the states the serving loop's byte-state kernel keeps for
// the best chain's replay (the packed-row kernels keep the state at the start
// of each slice only)
constexpr int kServeCheckpointEvery = 64;
// Register classes of the specialised serving kernels, named by their largest
// distance: d <= 15 but 9 (one word per row, eight wavefronts per SIMD), 17-21,
// 23-25, 27-29 and 31 (the largest kept apart to bound compile time).  d = 9
// has a class of its own: its sweep takes more registers than the others of
// the first class, and merged with them the kernel spills.  A serving slice
// makes one launch per class present.
constexpr int serve_class_max(int d)
{
    return d == 9 ? 9 : d <= 15 ? 15 : d <= 21 ? 21 : d <= 25 ? 25 : d <= 29 ? 29 : 31;
}

// Host-side lattice: geometry shared by every plan built on it.
struct Lattice {
    int layout = 0, d = 0, nq = 0, nstab = 0, per_class = 0;
    std::vector<int32_t> fq;      // [nstab][4], -1 absent
    std::vector<uint8_t> fm;      // [nstab][4] Pauli code of the generator on the slot
    std::vector<int32_t> fclass, fcolour, frank;
    std::vector<int32_t> fcx, fcy;  // face coordinates (rotated: cell (i,j); planar: doubled (x,y))
    std::vector<uint8_t> lx, lz;
    std::vector<int32_t> by_class;  // [4][per_class] face id
};

// Device-resident plan tables (one contiguous allocation) and their layout.
struct PlanDev {
    int nq, nstab, M, nblk;        // M generators per colour class, nblk = ceil(M/4)
    int ntypes, nranks, kneg;      // ranks [0, kneg) have dE <= 0
    int n_sweeps;
    int lanes;                     // lanes per chain (1..64)
    int layout, d;
    int row_words;                 // packed-row kernel: 32-bit words per lattice row (0 = unavailable)
    int rows;                      // packed-row kernels: rows of the grid (rotated d + 2, planar 2d - 1)
    int static_words;              // specialised kernel: words per unpadded row (0 = unavailable)
    int32_t W[4];
    const uint32_t *rowface;       // [4][4*nblk] row | bit offset << 8 | shape << 16 (packed-row kernel)
    const uint32_t *qpos;          // [nq] packed-row kernel: row << 8 | column of each qubit
    int ladder_k;                  // replica exchange: levels per ladder (0 = off)
    const uint32_t *ladder_thr;    // [ladder_k][nranks] acceptance thresholds of each level
    const uint64_t *ladder_pow;    // [32] fixed-point powers R_i of the exchange rule
    const Desc *desc;              // [4][M] by (class, rank)
    const Desc *face_desc;         // [nstab] by face id
    const uint8_t *lut;            // [ntypes][256] move-energy rank of a slot pattern
    const int32_t *dE;             // [nranks] ascending
    const uint32_t *thr;           // [n_sweeps][nranks]
    const uint8_t *lx, *lz;        // [nq]
    // greedy matching, per decoding-graph colour g
    int ncol[2];
    const int32_t *col_face[2];    // node -> face id (ascending)
    const int32_t *dint[2];        // [n][n] interior distance
    const int32_t *db[2];          // [n] boundary distance
    const int4 *adj[2];            // [n][4] (edge id, other node or -1, weight, 0), by edge id
};

struct Plan {
    Lattice lat;
    int32_t W[4], Wg[2];
    int n_sweeps = 0;
    std::vector<double> beta;
    std::vector<int32_t> dE;       // distinct move energies, ascending
    int kneg = 0;
    int ntypes = 0;
    int lanes_default = 1, lanes = 1;
    int row_words = 0;             // 0: the packed-row kernel does not apply to this lattice
    int use_rows = 0;              // 1: annealing runs on the packed-row kernel
    int static_d = 0;              // d if the packed-row kernel specialised to d applies, else 0
    int static_ok = 0;             // the plan's tables match the specialised schedule
    int static_words = 0;          // words per row of the specialised kernel's rows (2(d+1) bits)
    int order = 0;                 // XZZX_ORDER_COLOUR or XZZX_ORDER_RANDOM_SITE
    int planar_ok = 0;             // the planar kernel specialised to d applies
    int planar_d = 0;              // d while that kernel is in use, else 0
    int ladder_k = 0;              // replica exchange: levels per ladder (0 = off)
    double ladder_lo = 0, ladder_hi = 0;
    void *ladder_mem = nullptr;    // device tables of the ladder (thresholds per level, exchange powers)
    size_t lds_bytes_ladder() const;
    int nranks() const { return (int)dE.size(); }
    int device = 0;
    void *dmem = nullptr;          // device allocation holding every table
    size_t dbytes = 0;
    PlanDev hdev{};                // host copy with device pointers
    PlanDev *ddev = nullptr;       // device copy of hdev (inside dmem)
    size_t lds_bytes_anneal(int lanes) const;
    size_t lds_bytes_rows() const;
    size_t lds_bytes_site() const;
};


// Serving-loop task: consecutive chains of one resident request, all at the
// same sweep range (see k_serve_* in xzzx_kernels.hip).
struct ServeTask {
    const PlanDev *plan;
    const uint8_t *refs;     // request references [n_rep][nq]
    uint8_t *states;         // request chain states [4 n_rep][nq]
    int32_t *e3;             // request chain words [3][4 n_rep]: E, E_min, phase of E_min
    uint8_t *snap;           // replay: recovery destination [nq]
    const int32_t *best;     // replay: the request's best chain
    uint32_t uid;
    int32_t n_rep;
    int32_t chain0, nchains; // chains [chain0, chain0 + nchains) of the request
    int32_t t_begin, t_end;  // sweep range; t_begin == 0 starts from the references
    int32_t log_lanes;       // byte-state core: lanes per chain
    int32_t row_words;       // packed-row core: words per row
    uint8_t *cp;             // kept byte states [2][4 n_rep][nq] (nullable)
    uint32_t *cpk;           // kept packed rows [2][4 n_rep][cpk_words]
    int32_t *cpm;            // per chain: entry naming the replay start (see kept_entry)
    int32_t cpk_words;       // words per chain of a packed-rows buffer
};

// Serving-loop finish entry: per-coset reduction of one finished request,
// and where its result and recovery are gathered for the copy to the host.
struct ServeFinish {
    const int32_t *e3;       // request chain words [3][4 n_rep]
    const uint8_t *qraw;     // request raw symplectic bits [n_rep]
    int32_t *result;         // [8]: E_best, P*, best chain, unused, E_P[4]
    const uint8_t *recovery; // the request's recovery [nq] (written by the replay)
    uint8_t *out;            // gathered [32-byte result][nq recovery]
    int32_t n_rep;
    int32_t nq;
};

// One launch of a serving slice: tasks of one kernel family.
//   kind 0: packed-row kernel; 1: byte-state kernel; 2: packed-row kernel
//   specialised to distance d.
// One launch of a serving slice; the launches of a slice cover consecutive
// ranges of one device task array, starting at launches[0].tasks.
struct ServeLaunch {
    const ServeTask *tasks;
    int32_t n;
    int32_t kind;
    int32_t d;
    size_t lds;
};

int serve_greedy(const Plan &P, const uint8_t *d_syn, int64_t syn_stride, const uint32_t *d_uid,
                 const int32_t *d_slot_map, int n, int n_rep, uint8_t *refs_base, int64_t refs_stride,
                 uint8_t *qraw_base, int64_t qraw_stride, uint64_t seed, int mode, hipStream_t stream);
int serve_slice(const ServeLaunch *launches, int n_launches, uint64_t seed, hipStream_t stream);
// launch(i, s) for i < n: the first on `stream`, the others on side streams
// that wait for `stream`'s prior work; `stream` then waits for them all
int run_concurrently(hipStream_t stream, int n, const std::function<int(int, hipStream_t)> &launch);
int serve_finish(const ServeFinish *d_fin, const ServeTask *d_replay, int n, size_t lds_replay, uint64_t seed,
                 hipStream_t stream);

// ---- host helpers (xzzx_host.cpp) ----
void set_error(const std::string &msg);
int build_lattice(int layout, int d, Lattice &L);
int build_plan(const Lattice &L, const int32_t w[4], const int32_t wg[2], const double *beta,
               int n_sweeps, Plan &P);
uint32_t accept_threshold(double beta, int64_t dE);

}  // namespace xzzx

struct xzzx_lattice {
    xzzx::Lattice L;
};

struct xzzx_plan {
    xzzx::Plan P;
};
