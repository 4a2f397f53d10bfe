// orc_tree.cpp -- the oracle's block-based MR simulation (test infrastructure only).
//
// Plain FP64 transcription of the paper's method with a global time step:
//   * octree of fixed-size blocks (16^3 interior + 4 halo layers), addressed by Morton ids
//     with a headbit in a hash map (Sec. "Modular block-based MR algorithm");
//   * halo fill: copy from a same-level neighbour, else prediction from the parent
//     (eq:Prediction), external boundaries afterwards (periodic = wrap, zero-gradient);
//   * right-hand side from one numerical flux per face, with the coarse flux at a
//     resolution jump replaced by the average of the fine fluxes (algo:ComputeLoop,
//     coarse cell adjustment; applied every stage because the step is global);
//   * SSP-RK3 stages, CFL time step (eq:Cfl), conservative averaging of parents
//     (eq:Averaging) before every stage;
//   * after each step: details (eq:DetailFunction as u_l - P(u_{l-1})), level-wise
//     thresholds (eq:Thresholding, eq:LevelWiseEpsilon with D = 3), refine/coarsen;
//   * bottom-up initialisation of algo:Init (including level l_max);
//   * local time stepping (eq:LtsTimestep, algo:ComputeLoop, algo:Integration) as a
//     second step function, described where it is defined.
#include "orc.h"

#include <algorithm>
#include <omp.h>
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <vector>

namespace {

constexpr int P = ORC_P, H = ORC_H, N = ORC_IC;
constexpr int CELLS = P * P * P;
constexpr int ICELLS = N * N * N;
constexpr int PLANE = N * N;

inline int at(int q, int k, int j, int i) { return ((q * P + k) * P + j) * P + i; }
inline int ati(int q, int k, int j, int i) { return ((q * N + k) * N + j) * N + i; }

struct Block {
    int level = 0, bx = 0, by = 0, bz = 0;
    uint64_t id = 0;
    bool leaf = true;
    double detail = -1.0;
    int flag = 0;
    std::vector<double> u;     // 5 * 24^3 current (stage) state
    std::vector<double> u0;    // 5 * 16^3 state at t^n
    std::vector<double> rhs;   // 5 * 16^3
    std::vector<double> face[6];  // boundary face fluxes, 5 * 16 * 16 each
    // local time stepping only
    std::vector<double> F;        // 5 * 24^3 flux divergence (interior and halo)
    std::vector<double> u0p;      // 5 * 24^3 state at the start of the block's own step
    std::vector<double> acc[6];   // time-integrated boundary face fluxes, 5 * 16 * 16 each
    Block() : u(5 * CELLS, 0.0) {}
};

}  // namespace

struct orc_sim {
    orc_params p{};
    int shadow = 0;
    double time = 0.0;
    double llf_fraction = 0.0;
    int64_t lts_steps[ORC_MAX_LEVELS] = {};  // own steps completed per level (local time stepping)
    std::vector<double> fixed;   // conservative fixed-value halo states [6][lmax+1][4][5]
    std::unordered_map<uint64_t, Block *> map;
    std::vector<Block *> order;  // blocks sorted by (level, id); rebuilt after edits
    ~orc_sim() {
        for (auto &kv : map) delete kv.second;
    }
};

extern "C" {

// ------------------------------------------------------------------ Morton ids -------

uint64_t orc_morton_encode(int32_t shadow, int32_t level, int32_t bx, int32_t by, int32_t bz) {
    const int groups = shadow + level;
    uint64_t id = 1;  // headbit
    for (int g = groups - 1; g >= 0; --g) {
        const uint64_t x = (uint64_t)((bx >> g) & 1), y = (uint64_t)((by >> g) & 1),
                       z = (uint64_t)((bz >> g) & 1);
        id = (id << 3) | (z << 2) | (y << 1) | x;
    }
    return id;
}

static int id_groups(uint64_t id) {
    int msb = 63;
    while (msb > 0 && !((id >> msb) & 1ull)) --msb;
    return msb / 3;
}

int32_t orc_morton_level(uint64_t id, int32_t shadow) { return id_groups(id) - shadow; }

uint64_t orc_morton_neighbor(uint64_t id, int32_t d, int32_t dir, int32_t *wrapped) {
    // eq:NeigboorLookup: remove the headbit, walk every third bit of axis d from the
    // least significant group upwards, flipping until the carry (or borrow) stops.
    const int groups = id_groups(id);
    const int nbits = 3 * groups;
    const uint64_t head = 1ull << nbits;
    uint64_t n = id ^ head;
    int f = 0;
    for (int i = d; i < nbits; i += 3) {
        const int bit = (int)((n >> i) & 1ull);
        const int nb = !(bit ^ f);  // XNOR
        n = (n & ~(1ull << i)) | ((uint64_t)nb << i);
        f = (dir > 0) ? (nb | f) : ((!nb) | f);
    }
    if (wrapped) *wrapped = (f == 0);
    return n | head;
}

}  // extern "C"

namespace {

int level_extent(const orc_params &p, int axis, int level) { return p.n0[axis] << level; }

Block *find(orc_sim *s, int level, int bx, int by, int bz) {
    auto it = s->map.find(orc_morton_encode(s->shadow, level, bx, by, bz));
    return it == s->map.end() ? nullptr : it->second;
}

// Same-level neighbour position with external boundary handling.
// Returns false when the position lies outside a zero-gradient boundary.
bool neighbor_pos(const orc_sim *s, const Block *b, int dx, int dy, int dz, int out[3]) {
    const int d[3] = {dx, dy, dz};
    const int c[3] = {b->bx, b->by, b->bz};
    for (int a = 0; a < 3; ++a) {
        const int n = level_extent(s->p, a, b->level);
        int v = c[a] + d[a];
        if (v < 0 || v >= n) {
            if (s->p.bc[a] != 0) return false;
            v = (v + n) % n;
        }
        out[a] = v;
    }
    return true;
}

Block *parent_of(orc_sim *s, const Block *b) {
    if (b->level == 0) return nullptr;
    return find(s, b->level - 1, b->bx >> 1, b->by >> 1, b->bz >> 1);
}

Block *child_of(orc_sim *s, const Block *b, int ox, int oy, int oz) {
    return find(s, b->level + 1, 2 * b->bx + ox, 2 * b->by + oy, 2 * b->bz + oz);
}

void rebuild_order(orc_sim *s) {
    s->order.clear();
    for (auto &kv : s->map) s->order.push_back(kv.second);
    std::sort(s->order.begin(), s->order.end(), [](const Block *a, const Block *b) {
        if (a->level != b->level) return a->level < b->level;
        return a->id < b->id;
    });
}

std::vector<Block *> blocks_on_level(orc_sim *s, int level) {
    std::vector<Block *> v;
    for (Block *b : s->order)
        if (b->level == level) v.push_back(b);
    return v;
}

Block *add_block(orc_sim *s, int level, int bx, int by, int bz) {
    Block *b = new Block();
    b->level = level;
    b->bx = bx;
    b->by = by;
    b->bz = bz;
    b->id = orc_morton_encode(s->shadow, level, bx, by, bz);
    s->map[b->id] = b;
    return b;
}

double eps_level(const orc_params &p, int level) {
    // eq:LevelWiseEpsilon with D = 3.
    return std::ldexp(p.eps, -3 * (p.lmax - level));
}

double dx_level(const orc_params &p, int level) { return std::ldexp(p.dx0, -level); }

// ---------------------------------------------------------------- operators ----------

void predict_interior(const Block *parent, Block *child) {
    const int ox = child->bx & 1, oy = child->by & 1, oz = child->bz & 1;
    for (int q = 0; q < 5; ++q) {
        const double *pu = parent->u.data() + q * CELLS;
        for (int k = H; k < H + N; ++k)
            for (int j = H; j < H + N; ++j)
                for (int i = H; i < H + N; ++i)
                    child->u[at(q, k, j, i)] = orc_predict_cell(pu, ox, oy, oz, i, j, k);
    }
}

using Field = std::vector<double> Block::*;

void average_into_parent(orc_sim *s, Block *parent, Field fld = &Block::u) {
    for (int oz = 0; oz < 2; ++oz)
        for (int oy = 0; oy < 2; ++oy)
            for (int ox = 0; ox < 2; ++ox) {
                const Block *c = child_of(s, parent, ox, oy, oz);
                for (int q = 0; q < 5; ++q)
                    for (int K = 0; K < N / 2; ++K)
                        for (int J = 0; J < N / 2; ++J)
                            for (int I = 0; I < N / 2; ++I) {
                                double v[8];
                                for (int cz = 0; cz < 2; ++cz)
                                    for (int cy = 0; cy < 2; ++cy)
                                        for (int cx = 0; cx < 2; ++cx)
                                            v[cz * 4 + cy * 2 + cx] =
                                                (c->*fld)[at(q, H + 2 * K + cz, H + 2 * J + cy,
                                                             H + 2 * I + cx)];
                                (parent->*fld)[at(q, H + oz * N / 2 + K, H + oy * N / 2 + J,
                                                  H + ox * N / 2 + I)] = orc_average8(v);
                            }
            }
}

void project(orc_sim *s) {
    for (int l = s->p.lmax - 1; l >= 0; --l) {
        std::vector<Block *> lv = blocks_on_level(s, l);
#pragma omp parallel for schedule(static)
        for (long n = 0; n < (long)lv.size(); ++n)
            if (!lv[n]->leaf) average_into_parent(s, lv[n]);
    }
}

void fill_block_halos(orc_sim *s, Block *b, Field fld = &Block::u) {
    std::vector<double> &u = b->*fld;
    const int lo[3] = {0, H, H + N}, hi[3] = {H, H + N, P};
    Block *parent = parent_of(s, b);
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                int np[3];
                if (!neighbor_pos(s, b, dx, dy, dz, np)) continue;  // handled by the BC below
                const Block *nb = find(s, b->level, np[0], np[1], np[2]);
                for (int q = 0; q < 5; ++q)
                    for (int k = lo[dz + 1]; k < hi[dz + 1]; ++k)
                        for (int j = lo[dy + 1]; j < hi[dy + 1]; ++j)
                            for (int i = lo[dx + 1]; i < hi[dx + 1]; ++i) {
                                double v;
                                if (nb)
                                    v = (nb->*fld)[at(q, k - N * dz, j - N * dy, i - N * dx)];
                                else
                                    v = orc_predict_cell((parent->*fld).data() + q * CELLS,
                                                         b->bx & 1, b->by & 1, b->bz & 1, i, j, k);
                                u[at(q, k, j, i)] = v;
                            }
            }
    // External boundaries, axis by axis over the full padded extent: zero gradient (every
    // halo layer a copy of the boundary cell), symmetry (the halo the mirror image of the
    // interior, the momentum normal to the boundary reversed) or fixed values (each halo
    // layer the given state; the state field only: a flux-divergence field keeps its halo).
    const int c[3] = {b->bx, b->by, b->bz};
    for (int a = 0; a < 3; ++a) {
        if (s->p.bc[a] == 0) continue;
        const bool mirror = s->p.bc[a] == 2, fixed = s->p.bc[a] == 3;
        if (fixed && fld != &Block::u) continue;
        const int n = level_extent(s->p, a, b->level);
        for (int side = 0; side < 2; ++side) {
            if (side == 0 && c[a] != 0) continue;
            if (side == 1 && c[a] != n - 1) continue;
            for (int q = 0; q < 5; ++q)
                for (int h = 0; h < H; ++h) {
                    const int dst = side == 0 ? h : H + N + h;
                    const int src = mirror ? 2 * (side == 0 ? H : H + N) - 1 - dst : (side == 0 ? H : H + N - 1);
                    const double sign = mirror && q == 1 + a ? -1.0 : 1.0;
                    const int layer = side == 0 ? H - 1 - h : h;   // 0 at the face
                    const double fv = fixed ? s->fixed[(((2 * a + side) * (s->p.lmax + 1) + b->level) * 4 + layer) * 5 + q] : 0.0;
                    for (int m = 0; m < P; ++m)
                        for (int r = 0; r < P; ++r) {
                            int is[3], id[3];
                            is[a] = src;
                            id[a] = dst;
                            const int o1 = (a + 1) % 3, o2 = (a + 2) % 3;
                            is[o1] = id[o1] = r;
                            is[o2] = id[o2] = m;
                            u[at(q, id[2], id[1], id[0])] = fixed ? fv : sign * u[at(q, is[2], is[1], is[0])];
                        }
                }
        }
    }
}

void fill_halos(orc_sim *s, Field fld = &Block::u) {
    for (int l = 0; l <= s->p.lmax; ++l) {
        std::vector<Block *> lv = blocks_on_level(s, l);
#pragma omp parallel for schedule(static)
        for (long n = 0; n < (long)lv.size(); ++n) fill_block_halos(s, lv[n], fld);
    }
}

// Face fluxes of one leaf along all three axes and its right-hand side (without jump
// correction).  Returns the number of face-fields that used the LLF branch.
long block_rhs(const orc_sim *s, Block *b) {
    const double g = s->p.gamma, B = s->p.B;
    const double dx = dx_level(s->p, b->level);
    // F[d][q][m][r][f]: face f (0..16) along axis d; (r, m) = the other two interior
    // indices in increasing axis order.
    std::vector<double> F(3 * 5 * PLANE * (N + 1));
    auto fidx = [](int d, int q, int m, int r, int f) {
        return (((d * 5 + q) * N + m) * N + r) * (N + 1) + f;
    };
    long n_llf = 0;
    for (int d = 0; d < 3; ++d)
        for (int m = 0; m < N; ++m)
            for (int r = 0; r < N; ++r)
                for (int f = 0; f <= N; ++f) {
                    double st[30], Fh[5];
                    for (int j = 0; j < 6; ++j) {
                        const int along = f + 1 + j;  // padded index of stencil cell j
                        int c[3];
                        c[d] = along;
                        // the other two axes in increasing order: (o_lo, o_hi)
                        const int o_lo = d == 0 ? 1 : 0, o_hi = d == 2 ? 1 : 2;
                        c[o_lo] = H + r;
                        c[o_hi] = H + m;
                        for (int q = 0; q < 5; ++q) st[5 * j + q] = b->u[at(q, c[2], c[1], c[0])];
                    }
                    n_llf += s->p.eos == 1
                                 ? orc_tait_face_flux(d, st, g, B, s->p.tait_A, s->p.tait_rho0, Fh)
                                 : orc_face_flux_scheme(s->p.scheme, d, st, g, B, Fh);
                    if (s->p.mu > 0.0) {
                        // the two cells sharing the face and their tangential neighbours
                        const int o_lo = d == 0 ? 1 : 0, o_hi = d == 2 ? 1 : 2;
                        const int dn[5][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}};
                        double vs[50], Fv[5];
                        for (int sd = 0; sd < 2; ++sd)
                            for (int n = 0; n < 5; ++n) {
                                int c[3];
                                c[d] = H + f - 1 + sd;
                                c[o_lo] = H + r + dn[n][0];
                                c[o_hi] = H + m + dn[n][1];
                                for (int q = 0; q < 5; ++q) vs[(sd * 5 + n) * 5 + q] = b->u[at(q, c[2], c[1], c[0])];
                            }
                        orc_visc_face_flux(d, vs, s->p.mu, s->p.eos == 0, dx, Fv);
                        for (int q = 0; q < 5; ++q) Fh[q] -= Fv[q];
                    }
                    for (int q = 0; q < 5; ++q) F[fidx(d, q, m, r, f)] = Fh[q];
                }
    b->rhs.assign(5 * ICELLS, 0.0);
    for (int q = 0; q < 5; ++q)
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) {
                    const double ddx = F[fidx(0, q, k, j, i + 1)] - F[fidx(0, q, k, j, i)];
                    const double ddy = F[fidx(1, q, k, i, j + 1)] - F[fidx(1, q, k, i, j)];
                    const double ddz = F[fidx(2, q, j, i, k + 1)] - F[fidx(2, q, j, i, k)];
                    b->rhs[ati(q, k, j, i)] = -(ddx + ddy + ddz) / dx;
                }
    // Source term of eq:Euler: gravity, S(u) = (0, rho g, rho v . g), from the stage state.
    const double *gv = s->p.gravity;
    if (gv[0] != 0.0 || gv[1] != 0.0 || gv[2] != 0.0)
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) {
                    const double rho = b->u[at(0, H + k, H + j, H + i)];
                    double work = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        b->rhs[ati(1 + a, k, j, i)] += rho * gv[a];
                        work += b->u[at(1 + a, H + k, H + j, H + i)] * gv[a];
                    }
                    if (s->p.eos == 0) b->rhs[ati(4, k, j, i)] += work;   // Tait: energy not evolved
                }
    // Boundary face planes for the jump correction, stored [q][m][r].
    for (int side = 0; side < 6; ++side) {
        const int d = side / 2, f = (side % 2) ? N : 0;
        b->face[side].assign(5 * PLANE, 0.0);
        for (int q = 0; q < 5; ++q)
            for (int m = 0; m < N; ++m)
                for (int r = 0; r < N; ++r) b->face[side][(q * N + m) * N + r] = F[fidx(d, q, m, r, f)];
    }
    return n_llf;
}

// Face plane of block b on side `side`: its own flux if a leaf, else the area average of
// its children's planes on that side (recursively).
using Planes = std::vector<double>[6];

std::vector<double> face_plane(orc_sim *s, Block *b, int side, Planes Block::*pl = &Block::face) {
    if (b->leaf) return (b->*pl)[side];
    const int d = side / 2, hi = side % 2;
    const int o_lo = d == 0 ? 1 : 0, o_hi = d == 2 ? 1 : 2;
    std::vector<double> out(5 * PLANE, 0.0);
    for (int cm = 0; cm < 2; ++cm)
        for (int cr = 0; cr < 2; ++cr) {
            int o[3];
            o[d] = hi;
            o[o_lo] = cr;
            o[o_hi] = cm;
            Block *c = child_of(s, b, o[0], o[1], o[2]);
            const std::vector<double> cp = face_plane(s, c, side, pl);
            for (int q = 0; q < 5; ++q)
                for (int M = 0; M < N / 2; ++M)
                    for (int R = 0; R < N / 2; ++R) {
                        auto v = [&](int a, int bb) {
                            return cp[(q * N + 2 * M + bb) * N + 2 * R + a];
                        };
                        const double avg = ((v(0, 0) + v(1, 0)) + (v(0, 1) + v(1, 1))) / 4.0;
                        out[(q * N + cm * N / 2 + M) * N + cr * N / 2 + R] = avg;
                    }
        }
    return out;
}

// Replace the coarse flux at resolution jumps by the average of the fine fluxes.
void jump_correction(orc_sim *s, Block *b) {
    const double dx = dx_level(s->p, b->level);
    for (int side = 0; side < 6; ++side) {
        const int d = side / 2, hi = side % 2;
        int off[3] = {0, 0, 0};
        off[d] = hi ? 1 : -1;
        int np[3];
        if (!neighbor_pos(s, b, off[0], off[1], off[2], np)) continue;
        Block *nb = find(s, b->level, np[0], np[1], np[2]);
        if (!nb || nb->leaf) continue;
        const std::vector<double> fine = face_plane(s, nb, side ^ 1);
        const int o_lo = d == 0 ? 1 : 0, o_hi = d == 2 ? 1 : 2;
        for (int q = 0; q < 5; ++q)
            for (int m = 0; m < N; ++m)
                for (int r = 0; r < N; ++r) {
                    int c[3];
                    c[d] = hi ? N - 1 : 0;
                    c[o_lo] = r;
                    c[o_hi] = m;
                    const double own = b->face[side][(q * N + m) * N + r];
                    const double fn = fine[(q * N + m) * N + r];
                    const double corr = hi ? (own - fn) / dx : (fn - own) / dx;
                    b->rhs[ati(q, c[2], c[1], c[0])] += corr;
                }
    }
}

std::vector<Block *> leaves(orc_sim *s) {
    std::vector<Block *> v;
    for (Block *b : s->order)
        if (b->leaf) v.push_back(b);
    return v;
}

void compute_rhs(orc_sim *s) {
    std::vector<Block *> lv = leaves(s);
    long n_llf = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_llf)
    for (long n = 0; n < (long)lv.size(); ++n) n_llf += block_rhs(s, lv[n]);
    const double fields = (double)lv.size() * 3.0 * PLANE * (N + 1) * 5.0;
    s->llf_fraction = fields > 0 ? (double)n_llf / fields : 0.0;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < (long)lv.size(); ++n) jump_correction(s, lv[n]);
}

bool physical(const orc_sim *s, const Block *b) {
    for (int k = H; k < H + N; ++k)
        for (int j = H; j < H + N; ++j)
            for (int i = H; i < H + N; ++i) {
                double U[5];
                for (int q = 0; q < 5; ++q) U[q] = b->u[at(q, k, j, i)];
                if (s->p.eos == 1) {   // Tait: any positive density
                    if (!(U[0] > 0.0) || !std::isfinite(U[1] + U[2] + U[3])) return false;
                    continue;
                }
                const double p = orc_pressure(U, s->p.gamma, s->p.B);
                if (!(U[0] > 0.0) || !(p + s->p.B > 0.0) || !std::isfinite(U[4])) return false;
            }
    return true;
}

// eq:DetailFunction on the padded block: max over the 24^3 cells and q in {rho, E} of
// |u - P(u_parent)| / scale_q.
double detail_of(const double *u, const double *parent, int ox, int oy, int oz, double s_rho,
                 double s_E) {
    double d = 0.0;
    const int qs[2] = {0, 4};
    const double sc[2] = {s_rho, s_E};
    for (int n = 0; n < 2; ++n) {
        const int q = qs[n];
        const double *pu = parent + q * CELLS;
        for (int k = 0; k < P; ++k)
            for (int j = 0; j < P; ++j)
                for (int i = 0; i < P; ++i) {
                    const double pred = orc_predict_cell(pu, ox, oy, oz, i, j, k);
                    const double v = std::fabs(u[at(q, k, j, i)] - pred) / sc[n];
                    d = std::max(d, v);
                }
    }
    return d;
}

double block_detail(orc_sim *s, Block *b) {
    Block *par = parent_of(s, b);
    return detail_of(b->u.data(), par->u.data(), b->bx & 1, b->by & 1, b->bz & 1, s->p.scale_rho,
                     s->p.scale_E);
}

void compute_details(orc_sim *s) {
    std::vector<Block *> all = s->order;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < (long)all.size(); ++n)
        all[n]->detail = all[n]->level == 0 ? -1.0 : block_detail(s, all[n]);
}

// Refine/keep/coarsen decision for every leaf (non-leaves get 2).
void compute_flags(orc_sim *s) {
    for (Block *b : s->order) {
        if (!b->leaf) { b->flag = 2; continue; }
        const int l = b->level;
        if (l < s->p.lmax && b->detail >= eps_level(s->p, l)) { b->flag = 1; continue; }
        b->flag = 0;
        if (l < 2) continue;
        Block *par = parent_of(s, b);
        bool all_small = true;
        for (int o = 0; o < 8 && all_small; ++o) {
            const Block *c = child_of(s, par, o & 1, (o >> 1) & 1, o >> 2);
            if (!c->leaf || !(c->detail < eps_level(s->p, l))) all_small = false;
        }
        if (all_small && par->detail < eps_level(s->p, l - 1)) b->flag = -1;
    }
}

void refine(orc_sim *s, Block *b) {
    for (int o = 0; o < 8; ++o) {
        Block *c = add_block(s, b->level + 1, 2 * b->bx + (o & 1), 2 * b->by + ((o >> 1) & 1),
                             2 * b->bz + (o >> 2));
        predict_interior(b, c);
    }
    b->leaf = false;
}

void coarsen(orc_sim *s, Block *par) {
    for (int o = 0; o < 8; ++o) {
        Block *c = child_of(s, par, o & 1, (o >> 1) & 1, o >> 2);
        s->map.erase(c->id);
        delete c;
    }
    par->leaf = true;
}

void commit_flags(orc_sim *s) {
    std::vector<Block *> to_refine, to_coarsen;
    for (Block *b : s->order) {
        if (b->flag == 1) to_refine.push_back(b);
        if (b->flag == -1 && (b->bx & 1) == 0 && (b->by & 1) == 0 && (b->bz & 1) == 0)
            to_coarsen.push_back(parent_of(s, b));
    }
    for (Block *b : to_refine) refine(s, b);
    for (Block *b : to_coarsen) coarsen(s, b);
    rebuild_order(s);
}

// ------------------------------------------------------------ local time stepping ----
//
// eq:LtsTimestep: level l advances with its own step dt_l = 2^(lmax - l) dt, dt being the
// eq:Cfl step of level lmax; a macro step is 2^lmax micro steps r (algo:ComputeLoop).
// Level l completes one step of its own at micro step r when r + 1 is a multiple of
// 2^(lmax - l); the levels doing so form the active set {lmax, ..., lmax + 1 -
// popcount((r + 1) xor r)} of algo:ComputeLoop.  A level's first stage is evaluated at the
// micro step its step starts in, its integration (all stages) happens at the micro step it
// ends in.  Halo cells at a resolution jump carry their own state, integrated with the
// flux divergence predicted from the coarser level (algo:Integration); the flux divergence
// is averaged into parents and predicted into halos like the conserved variables.
// Conservation: every leaf sums its boundary face fluxes over its stages and steps,
// weighted as the RK scheme weights them; at the last stage of its step a coarse leaf
// next to a refined same-level neighbour replaces its own sum on that face by the area
// average of the fine sums (the coarse cell adjustment of algo:ComputeLoop).

// Lowest level that ends a step at micro step r.
int lts_lowest_ending(int lmax, int r) {
    return lmax + 1 - __builtin_popcount((unsigned)((r + 1) ^ r));
}

// Lowest level that starts a step at micro step r (every level at r = 0).
int lts_lowest_starting(int lmax, int r) { return r == 0 ? 0 : lts_lowest_ending(lmax, r - 1); }

enum FaceKind { FACE_PRESENT, FACE_BOUNDARY, FACE_JUMP };

FaceKind face_kind(orc_sim *s, const Block *b, int side, Block **nb_out = nullptr) {
    int off[3] = {0, 0, 0};
    off[side >> 1] = (side & 1) ? 1 : -1;
    int np[3];
    if (!neighbor_pos(s, b, off[0], off[1], off[2], np)) return FACE_BOUNDARY;
    Block *nb = find(s, b->level, np[0], np[1], np[2]);
    if (nb_out) *nb_out = nb;
    return nb ? FACE_PRESENT : FACE_JUMP;
}

// Level of the leaf on the other side of a face: the block's own level unless the face is
// a resolution jump, then the level of the coarser leaf that covers the position.
int across_level(orc_sim *s, const Block *b, int side) {
    if (face_kind(s, b, side) != FACE_JUMP) return b->level;
    int off[3] = {0, 0, 0};
    off[side >> 1] = (side & 1) ? 1 : -1;
    int np[3];
    neighbor_pos(s, b, off[0], off[1], off[2], np);
    for (int m = b->level - 1; m >= 0; --m) {
        const int sh = b->level - m;
        if (find(s, m, np[0] >> sh, np[1] >> sh, np[2] >> sh)) return m;
    }
    return 0;
}

// The three halo layers of a face that the flux stencils read, interior extent across.
template <class Fn>
void for_face_slab(int side, Fn fn) {
    const int d = side >> 1, hi = side & 1;
    const int o_lo = d == 0 ? 1 : 0, o_hi = d == 2 ? 1 : 2;
    for (int h = 0; h < 3; ++h)
        for (int m = H; m < H + N; ++m)
            for (int r = H; r < H + N; ++r) {
                int c[3];
                c[d] = hi ? H + N + h : H - 3 + h;
                c[o_lo] = r;
                c[o_hi] = m;
                fn(c[2], c[1], c[0]);
            }
}

// State halos of a leaf that are copies (same-level neighbour) or an external boundary
// (zero gradient, symmetry, fixed values, as in fill_block_halos); faces at resolution
// jumps keep their integrated values.
void fill_present_faces(orc_sim *s, Block *b) {
    for (int side = 0; side < 6; ++side) {
        Block *nb = nullptr;
        const FaceKind kind = face_kind(s, b, side, &nb);
        if (kind == FACE_JUMP) continue;
        const int d = side >> 1, hi = side & 1, bc = s->p.bc[d];
        int off[3] = {0, 0, 0};
        off[d] = hi ? 1 : -1;
        for (int q = 0; q < 5; ++q)
            for_face_slab(side, [&](int k, int j, int i) {
                if (kind == FACE_PRESENT) {
                    b->u[at(q, k, j, i)] = nb->u[at(q, k - N * off[2], j - N * off[1], i - N * off[0])];
                    return;
                }
                int c[3] = {i, j, k};
                const int dst = c[d];
                if (bc == 3) {
                    const int layer = hi ? dst - (H + N) : H - 1 - dst;
                    b->u[at(q, k, j, i)] = s->fixed[((side * (s->p.lmax + 1) + b->level) * 4 + layer) * 5 + q];
                    return;
                }
                c[d] = bc == 2 ? 2 * (hi ? H + N : H) - 1 - dst : (hi ? H + N - 1 : H);
                const double sign = bc == 2 && q == 1 + d ? -1.0 : 1.0;
                b->u[at(q, k, j, i)] = sign * b->u[at(q, c[2], c[1], c[0])];
            });
    }
}

// One RK stage of a leaf's own step (algo:Integration): interior cells and the halo cells
// of its resolution-jump faces, from the stored flux divergence; the boundary face fluxes
// of the stage are added to the leaf's sums with the stage's weight in the RK scheme
// (SSP-RK3: 1/6, 1/6, 2/3).
void lts_integrate(orc_sim *s, Block *b, int st, double dtl) {
    static const double bw[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
    if (st == 0) b->u0p = b->u;
    auto upd = [&](int q, int k, int j, int i) {
        const int n = at(q, k, j, i);
        b->u[n] = orc_ssprk3_stage(st, b->u0p[n], b->u[n], b->F[n], dtl);
    };
    for (int q = 0; q < 5; ++q)
        for (int k = H; k < H + N; ++k)
            for (int j = H; j < H + N; ++j)
                for (int i = H; i < H + N; ++i) upd(q, k, j, i);
    for (int side = 0; side < 6; ++side) {
        if (face_kind(s, b, side) == FACE_JUMP)
            for (int q = 0; q < 5; ++q)
                for_face_slab(side, [&](int k, int j, int i) { upd(q, k, j, i); });
        for (int n = 0; n < 5 * PLANE; ++n) b->acc[side][n] += bw[st] * dtl * b->face[side][n];
    }
}

// Coarse cell adjustment at the end of a coarse leaf's step: on faces whose same-level
// neighbour is refined, the own time-integrated flux is replaced by the average of the
// fine ones.
void lts_adjust(orc_sim *s, Block *b) {
    const double dx = dx_level(s->p, b->level);
    for (int side = 0; side < 6; ++side) {
        Block *nb = nullptr;
        if (face_kind(s, b, side, &nb) != FACE_PRESENT || nb->leaf) continue;
        const std::vector<double> fine = face_plane(s, nb, side ^ 1, &Block::acc);
        const int d = side >> 1, hi = side & 1;
        const int o_lo = d == 0 ? 1 : 0, o_hi = d == 2 ? 1 : 2;
        for (int q = 0; q < 5; ++q)
            for (int m = 0; m < N; ++m)
                for (int r = 0; r < N; ++r) {
                    int c[3];
                    c[d] = hi ? H + N - 1 : H;
                    c[o_lo] = H + r;
                    c[o_hi] = H + m;
                    const double own = b->acc[side][(q * N + m) * N + r];
                    const double fn = fine[(q * N + m) * N + r];
                    b->u[at(q, c[2], c[1], c[0])] += hi ? (own - fn) / dx : (fn - own) / dx;
                }
    }
}

// Parents of the blocks on levels >= lo (descending), from their children.
void average_levels(orc_sim *s, int lo, Field fld) {
    for (int l = s->p.lmax; l >= std::max(lo, 1); --l) {
        std::vector<Block *> pv = blocks_on_level(s, l - 1);
#pragma omp parallel for schedule(static)
        for (long n = 0; n < (long)pv.size(); ++n)
            if (!pv[n]->leaf) average_into_parent(s, pv[n], fld);
    }
}

void adapt_tree(orc_sim *s) {
    project(s);
    fill_halos(s);
    compute_details(s);
    compute_flags(s);
    commit_flags(s);
}

int lts_macro_step(orc_sim *s, double dt) {
    const int lmax = s->p.lmax;
    project(s);
    fill_halos(s);
    for (Block *b : s->order) {
        b->F.assign(5 * CELLS, 0.0);
        for (int side = 0; side < 6; ++side) b->acc[side].assign(5 * PLANE, 0.0);
    }
    const std::vector<Block *> lv = leaves(s);
    for (int r = 0; r < (1 << lmax); ++r) {
        const int lo_end = lts_lowest_ending(lmax, r);
        std::vector<Block *> ending;
        for (Block *b : lv)
            if (b->level >= lo_end) ending.push_back(b);
        for (int st = 0; st < 3; ++st) {
            const int lo_rhs = st == 0 ? lts_lowest_starting(lmax, r) : lo_end;
            std::vector<Block *> eval;
            for (Block *b : lv)
                if (b->level >= lo_rhs) eval.push_back(b);
#pragma omp parallel for schedule(static)
            for (long n = 0; n < (long)eval.size(); ++n) fill_present_faces(s, eval[n]);
#pragma omp parallel for schedule(static)
            for (long n = 0; n < (long)eval.size(); ++n) {
                Block *b = eval[n];
                block_rhs(s, b);
                for (int q = 0; q < 5; ++q)
                    for (int k = 0; k < N; ++k)
                        for (int j = 0; j < N; ++j)
                            for (int i = 0; i < N; ++i)
                                b->F[at(q, H + k, H + j, H + i)] = b->rhs[ati(q, k, j, i)];
            }
            average_levels(s, lo_rhs, &Block::F);
            fill_halos(s, &Block::F);
            int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
            for (long n = 0; n < (long)ending.size(); ++n) {
                Block *b = ending[n];
                lts_integrate(s, b, st, std::ldexp(dt, lmax - b->level));
                if (!physical(s, b)) bad += 1;
            }
            if (bad) return -5;
            if (st == 2) {
#pragma omp parallel for schedule(static)
                for (long n = 0; n < (long)ending.size(); ++n) lts_adjust(s, ending[n]);
                // the sums a coarse leaf has just used start again
                for (Block *b : lv)
                    for (int side = 0; side < 6; ++side)
                        if (across_level(s, b, side) >= lo_end) std::fill(b->acc[side].begin(), b->acc[side].end(), 0.0);
                for (int l = lo_end; l <= lmax; ++l) s->lts_steps[l] += 1;
            }
            average_levels(s, lo_end, &Block::u);
        }
    }
    return 0;
}

void impose_ic(orc_sim *s, Block *b, orc_ic_fn ic, void *user) {
    std::vector<double> prim(5 * ICELLS);
    ic(user, b->level, b->bx, b->by, b->bz, prim.data());
    const double g = s->p.gamma, B = s->p.B;
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                const double rho = prim[ati(0, k, j, i)], u = prim[ati(1, k, j, i)],
                             v = prim[ati(2, k, j, i)], w = prim[ati(3, k, j, i)],
                             p = prim[ati(4, k, j, i)];
                b->u[at(0, H + k, H + j, H + i)] = rho;
                b->u[at(1, H + k, H + j, H + i)] = rho * u;
                b->u[at(2, H + k, H + j, H + i)] = rho * v;
                b->u[at(3, H + k, H + j, H + i)] = rho * w;
                // Tait: the pressure follows from the density; the energy is not evolved
                b->u[at(4, H + k, H + j, H + i)] =
                    s->p.eos == 1 ? 0.0 : (p + g * B) / (g - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
            }
}

}  // namespace

extern "C" {

orc_sim *orc_sim_create(const orc_params *p) {
    orc_sim *s = new orc_sim();
    s->p = *p;
    s->p.bc_fixed = nullptr;
    if (p->bc_fixed) {
        // stored conservative, converted with the EOS like the initial condition
        const int nl = p->lmax + 1;
        s->fixed.assign((size_t)6 * nl * 4 * 5, 0.0);
        const double g = p->gamma, B = p->B;
        for (int n = 0; n < 6 * nl * 4; ++n) {
            const double *w = p->bc_fixed + 5 * n;
            double *u = s->fixed.data() + 5 * n;
            u[0] = w[0];
            for (int a = 0; a < 3; ++a) u[1 + a] = w[0] * w[1 + a];
            u[4] = p->eos == 1 ? 0.0
                               : (w[4] + g * B) / (g - 1.0) + 0.5 * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
        }
    }
    int mx = std::max(p->n0[0], std::max(p->n0[1], p->n0[2]));
    while ((1 << s->shadow) < mx) ++s->shadow;
    return s;
}

void orc_sim_free(orc_sim *s) { delete s; }

int orc_sim_init(orc_sim *s, orc_ic_fn ic, void *user) {
    for (int z = 0; z < s->p.n0[2]; ++z)
        for (int y = 0; y < s->p.n0[1]; ++y)
            for (int x = 0; x < s->p.n0[0]; ++x) impose_ic(s, add_block(s, 0, x, y, z), ic, user);
    rebuild_order(s);
    for (int m = 1; m <= s->p.lmax; ++m) {
        std::vector<Block *> parents = blocks_on_level(s, m - 1);
        std::vector<Block *> fresh;
        for (Block *b : parents) {
            for (int o = 0; o < 8; ++o)
                fresh.push_back(add_block(s, m, 2 * b->bx + (o & 1), 2 * b->by + ((o >> 1) & 1),
                                          2 * b->bz + (o >> 2)));
            b->leaf = false;
        }
        for (Block *c : fresh) impose_ic(s, c, ic, user);
        rebuild_order(s);
        if (m > 1) {
            fill_halos(s);
            std::vector<Block *> lv = blocks_on_level(s, m);
#pragma omp parallel for schedule(static)
            for (long n = 0; n < (long)lv.size(); ++n) lv[n]->detail = block_detail(s, lv[n]);
            const double eps = eps_level(s->p, m);
            std::vector<Block *> drop;
            for (Block *b : parents) {
                bool small = true;
                for (int o = 0; o < 8; ++o)
                    if (!(child_of(s, b, o & 1, (o >> 1) & 1, o >> 2)->detail < eps)) small = false;
                if (small) drop.push_back(b);
            }
            for (Block *b : drop) coarsen(s, b);
            rebuild_order(s);
        }
    }
    project(s);
    for (Block *b : s->order)
        if (!physical(s, b)) return -5;
    return 0;
}

double orc_sim_dt(const orc_sim *s) {
    double mx[3] = {0.0, 0.0, 0.0};
    for (const Block *b : s->order) {
        if (!b->leaf) continue;
        for (int k = H; k < H + N; ++k)
            for (int j = H; j < H + N; ++j)
                for (int i = H; i < H + N; ++i) {
                    double U[5];
                    for (int q = 0; q < 5; ++q) U[q] = b->u[at(q, k, j, i)];
                    const double c =
                        s->p.eos == 1 ? orc_tait_sound_speed(U[0], s->p.gamma, s->p.B, s->p.tait_rho0)
                                      : std::sqrt(s->p.gamma * (orc_pressure(U, s->p.gamma, s->p.B) + s->p.B) / U[0]);
                    for (int a = 0; a < 3; ++a)
                        mx[a] = std::max(mx[a], std::fabs(U[1 + a] / U[0]) + c);
                }
    }
    // eq:Cfl sums the three directional maxima; they are added in ascending order so that
    // dt does not depend on which axis is called x (a rotated problem gets the same dt)
    std::sort(mx, mx + 3);
    const double dx = dx_level(s->p, s->p.lmax);
    const double dt = s->p.cfl * dx / ((mx[0] + mx[1]) + mx[2]);
    if (!(s->p.mu > 0.0)) return dt;
    // with viscosity, also the explicit bound of the viscous terms at the smallest density
    double rinv = 0.0;
    for (const Block *b : s->order) {
        if (!b->leaf) continue;
        for (int k = H; k < H + N; ++k)
            for (int j = H; j < H + N; ++j)
                for (int i = H; i < H + N; ++i) rinv = std::max(rinv, 1.0 / b->u[at(0, k, j, i)]);
    }
    return std::min(dt, orc_visc_dt(s->p.cfl, dx, s->p.mu, rinv));
}

double orc_ssprk3_stage(int stage, double u0, double us, double L, double dt) {
    const double a[3] = {1.0, 0.25, 2.0 / 3.0};
    return u0 + a[stage] * ((us - u0) + dt * L);
}

int orc_sim_step(orc_sim *s, double *dt_out) {
    const double dt = orc_sim_dt(s);
    if (dt_out) *dt_out = dt;
    return orc_sim_step_dt(s, dt);
}

int orc_sim_step_dt(orc_sim *s, double dt) {
    std::vector<Block *> lv = leaves(s);
    for (Block *b : lv) {
        b->u0.assign(5 * ICELLS, 0.0);
        for (int q = 0; q < 5; ++q)
            for (int k = 0; k < N; ++k)
                for (int j = 0; j < N; ++j)
                    for (int i = 0; i < N; ++i)
                        b->u0[ati(q, k, j, i)] = b->u[at(q, H + k, H + j, H + i)];
    }
    int bad = 0;
    for (int st = 0; st < 3; ++st) {
        project(s);
        fill_halos(s);
        compute_rhs(s);
#pragma omp parallel for schedule(static) reduction(+ : bad)
        for (long n = 0; n < (long)lv.size(); ++n) {
            Block *b = lv[n];
            for (int q = 0; q < 5; ++q)
                for (int k = 0; k < N; ++k)
                    for (int j = 0; j < N; ++j)
                        for (int i = 0; i < N; ++i) {
                            const double u0 = b->u0[ati(q, k, j, i)];
                            double &u = b->u[at(q, H + k, H + j, H + i)];
                            u = orc_ssprk3_stage(st, u0, u, b->rhs[ati(q, k, j, i)], dt);
                        }
            if (!physical(s, b)) bad += 1;
        }
        if (bad) return -5;
    }
    s->time += dt;
    if (s->p.adapt) {
        project(s);
        fill_halos(s);
        compute_details(s);
        compute_flags(s);
        commit_flags(s);
    }
    return 0;
}

int orc_sim_step_lts(orc_sim *s, double *dt_out) {
    const double dt = orc_sim_dt(s);
    if (dt_out) *dt_out = dt;
    return orc_sim_step_lts_dt(s, dt);
}

int orc_sim_step_lts_dt(orc_sim *s, double dt) {
    // the viscous fluxes read edge halos, which the local time stepping here does not keep
    if (s->p.mu > 0.0) return -1;
    const int rc = lts_macro_step(s, dt);
    if (rc) return rc;
    s->time += std::ldexp(dt, s->p.lmax);
    if (s->p.adapt) adapt_tree(s);
    return 0;
}

void orc_sim_lts_steps(const orc_sim *s, int64_t *out) {
    for (int l = 0; l < ORC_MAX_LEVELS; ++l) out[l] = s->lts_steps[l];
}

int32_t orc_lts_lowest_ending(int32_t lmax, int32_t r) { return lts_lowest_ending(lmax, r); }

int32_t orc_sim_nblocks(const orc_sim *s) { return (int32_t)s->order.size(); }

void orc_sim_blocks(const orc_sim *s, int64_t *info) {
    for (size_t n = 0; n < s->order.size(); ++n) {
        const Block *b = s->order[n];
        int64_t *r = info + 8 * n;
        r[0] = b->level;
        r[1] = b->bx;
        r[2] = b->by;
        r[3] = b->bz;
        r[4] = b->leaf ? 1 : 0;
        r[5] = b->flag;
        r[6] = (int64_t)b->id;
        r[7] = 0;
    }
}

void orc_sim_get_block(const orc_sim *s, int32_t idx, double *out) {
    std::memcpy(out, s->order[idx]->u.data(), sizeof(double) * 5 * CELLS);
}

void orc_sim_set_block(orc_sim *s, int32_t idx, const double *in) {
    std::memcpy(s->order[idx]->u.data(), in, sizeof(double) * 5 * CELLS);
}

double orc_sim_detail(const orc_sim *s, int32_t idx) { return s->order[idx]->detail; }

void orc_block_rhs(const double *u_padded, double gamma, double B, double dx, double *L) {
    orc_block_rhs_scheme(0, u_padded, gamma, B, dx, L);
}

void orc_block_rhs_scheme(int scheme, const double *u_padded, double gamma, double B, double dx,
                          double *L) {
    orc_sim tmp;
    tmp.p.scheme = scheme;
    tmp.p.gamma = gamma;
    tmp.p.B = B;
    tmp.p.dx0 = dx;
    Block b;
    b.level = 0;
    b.u.assign(u_padded, u_padded + 5 * CELLS);
    block_rhs(&tmp, &b);
    std::memcpy(L, b.rhs.data(), sizeof(double) * 5 * ICELLS);
}

double orc_block_detail(const double *u_padded, const double *parent_padded, int ox, int oy, int oz,
                        double s_rho, double s_E) {
    return detail_of(u_padded, parent_padded, ox, oy, oz, s_rho, s_E);
}

int orc_sim_refine(orc_sim *s, int32_t level, int32_t bx, int32_t by, int32_t bz) {
    Block *b = find(s, level, bx, by, bz);
    if (!b || !b->leaf || level >= s->p.lmax) return -1;
    fill_halos(s);  // the prediction reads the parent's halos
    refine(s, b);
    rebuild_order(s);
    return 0;
}

int orc_sim_coarsen(orc_sim *s, int32_t level, int32_t bx, int32_t by, int32_t bz) {
    Block *b = find(s, level, bx, by, bz);
    if (!b || b->leaf) return -1;
    for (int o = 0; o < 8; ++o)
        if (!child_of(s, b, o & 1, (o >> 1) & 1, o >> 2)->leaf) return -1;
    coarsen(s, b);
    rebuild_order(s);
    return 0;
}

void orc_sim_project(orc_sim *s) { project(s); }
void orc_sim_fill_halos(orc_sim *s) { fill_halos(s); }

int32_t orc_sim_rhs(orc_sim *s, double *L_out) {
    compute_rhs(s);
    int32_t n = 0;
    for (Block *b : s->order) {
        if (!b->leaf) continue;
        if (L_out) std::memcpy(L_out + (size_t)n * 5 * ICELLS, b->rhs.data(), sizeof(double) * 5 * ICELLS);
        ++n;
    }
    return n;
}

void orc_sim_details(orc_sim *s, double *det_out, int8_t *flag_out) {
    compute_details(s);
    compute_flags(s);
    for (size_t n = 0; n < s->order.size(); ++n) {
        if (det_out) det_out[n] = s->order[n]->detail;
        if (flag_out) flag_out[n] = (int8_t)s->order[n]->flag;
    }
}

void orc_sim_totals(const orc_sim *s, double *tot) {
    for (int q = 0; q < 5; ++q) tot[q] = 0.0;
    for (const Block *b : s->order) {
        if (!b->leaf) continue;
        const double dx = dx_level(s->p, b->level);
        const double vol = dx * dx * dx;
        for (int q = 0; q < 5; ++q) {
            double sum = 0.0;
            for (int k = H; k < H + N; ++k)
                for (int j = H; j < H + N; ++j)
                    for (int i = H; i < H + N; ++i) sum += b->u[at(q, k, j, i)];
            tot[q] += sum * vol;
        }
    }
}

double orc_sim_time(const orc_sim *s) { return s->time; }
double orc_sim_llf_fraction(const orc_sim *s) { return s->llf_fraction; }

int orc_num_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
