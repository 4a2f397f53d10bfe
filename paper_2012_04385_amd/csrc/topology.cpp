// topology.cpp -- host-side octree of fixed-size blocks.
//
// Light-weight topology separated from the heavy block data (Sec. "Modular block-based
// MR algorithm" and "Algorithm and Implementation"): nodes are identified by Morton ids
// with a headbit and found through a hash map; the device only ever sees slot indices
// and the tables built here (per-slot metadata, children, 27-entry same-level
// neighbourhood, and work lists grouped by level).
#include <algorithm>

#include "mrfv_internal.h"

namespace mrfv {

// Spread the low 21 bits of v so that bit i lands at bit 3i.
static uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

static uint64_t compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return v;
}

uint64_t morton_encode(int shadow, int level, int bx, int by, int bz) {
    const int groups = shadow + level;
    const uint64_t body = spread3((uint64_t)bx) | (spread3((uint64_t)by) << 1) |
                          (spread3((uint64_t)bz) << 2);
    return (1ull << (3 * groups)) | body;
}

uint64_t Topology::key(int inst, int level, int bx, int by, int bz) {
    // 12 bits instance, 4 bits level, 16 bits per coordinate
    return ((uint64_t)inst << 52) | ((uint64_t)level << 48) | ((uint64_t)bz << 32) |
           ((uint64_t)by << 16) | (uint64_t)bx;
}

void Topology::reset(int capacity, const std::vector<mrfv_instance> &inst) {
    blocks_.assign(capacity, HostBlock());
    free_.clear();
    for (int s = capacity - 1; s >= 0; --s) free_.push_back(s);
    map_.clear();
    map_.reserve(2 * capacity);
    inst_ = inst;
    shadow_.clear();
    for (const auto &p : inst) {
        int m = std::max(p.n0[0], std::max(p.n0[1], p.n0[2])), s = 0;
        while ((1 << s) < m) ++s;
        shadow_.push_back(s);
    }
    n_alive_ = 0;
}

int Topology::add_block(int inst, int level, int bx, int by, int bz) {
    if (free_.empty()) return -1;
    const int s = free_.back();
    free_.pop_back();
    HostBlock &b = blocks_[s];
    b = HostBlock();
    b.inst = inst;
    b.level = level;
    b.bx = bx;
    b.by = by;
    b.bz = bz;
    b.alive = true;
    b.leaf = true;
    b.morton = morton_encode(shadow_[inst], level, bx, by, bz);
    if (level > 0) b.parent = find(inst, level - 1, bx >> 1, by >> 1, bz >> 1);
    map_[key(inst, level, bx, by, bz)] = s;
    ++n_alive_;
    return s;
}

int Topology::find(int inst, int level, int bx, int by, int bz) const {
    auto it = map_.find(key(inst, level, bx, by, bz));
    return it == map_.end() ? -1 : it->second;
}

bool Topology::refine(int slot, std::vector<int> *created) {
    if ((int)free_.size() < 8) return false;
    HostBlock &b = blocks_[slot];
    for (int o = 0; o < 8; ++o) {
        const int c = add_block(b.inst, b.level + 1, 2 * b.bx + (o & 1), 2 * b.by + ((o >> 1) & 1),
                                2 * b.bz + (o >> 2));
        blocks_[slot].child[o] = c;
        if (created) created->push_back(c);
    }
    blocks_[slot].leaf = false;
    return true;
}

void Topology::remove_block(int s) {
    HostBlock &b = blocks_[s];
    map_.erase(key(b.inst, b.level, b.bx, b.by, b.bz));
    b.alive = false;
    free_.push_back(s);
    --n_alive_;
}

void Topology::coarsen(int p) {
    for (int o = 0; o < 8; ++o) {
        remove_block(blocks_[p].child[o]);
        blocks_[p].child[o] = -1;
    }
    blocks_[p].leaf = true;
}

bool Topology::commit(const int8_t *flags, std::vector<TreeOp> *ops, std::vector<int> *fresh) {
    std::vector<int> order = alive_sorted();
    std::vector<int> coarsen_p, refine_s;
    for (int s : order) {
        const HostBlock &b = blocks_[s];
        if (!b.leaf) continue;
        if (flags[s] == 1) refine_s.push_back(s);
        if (flags[s] == -1 && (b.bx & 1) == 0 && (b.by & 1) == 0 && (b.bz & 1) == 0)
            coarsen_p.push_back(b.parent);
    }
    // all or nothing: every refinement needs 8 free slots, counting the slots the
    // coarsenings free first, so a commit that cannot complete leaves the tree unchanged
    if ((int64_t)free_.size() + 8 * (int64_t)coarsen_p.size() < 8 * (int64_t)refine_s.size())
        return false;
    for (int p : coarsen_p) {
        TreeOp op{-1, p, {}};
        for (int o = 0; o < 8; ++o) op.child[o] = blocks_[p].child[o];
        coarsen(p);
        if (ops) ops->push_back(op);
    }
    std::vector<int> created;
    for (int s : refine_s) {
        created.clear();
        if (!refine(s, &created)) return false;
        TreeOp op{1, s, {}};
        for (int o = 0; o < 8; ++o) op.child[o] = created[o];
        if (ops) ops->push_back(op);
        if (fresh) fresh->insert(fresh->end(), created.begin(), created.end());
    }
    return true;
}

void Topology::undo(const std::vector<TreeOp> &ops) {
    for (auto it = ops.rbegin(); it != ops.rend(); ++it) {
        const TreeOp &op = *it;
        HostBlock &p = blocks_[op.slot];
        if (op.kind == 1) {
            // remove the children newest first: the free list regains its order
            for (int o = 7; o >= 0; --o) remove_block(op.child[o]);
            for (int o = 0; o < 8; ++o) p.child[o] = -1;
            p.leaf = true;
        } else {
            // re-create the removed children in their slots (the last freed comes back first)
            for (int o = 7; o >= 0; --o) {
                const int s = free_.back();
                free_.pop_back();
                HostBlock &c = blocks_[s];
                c = HostBlock();
                c.inst = p.inst;
                c.level = p.level + 1;
                c.bx = 2 * p.bx + (o & 1);
                c.by = 2 * p.by + ((o >> 1) & 1);
                c.bz = 2 * p.bz + (o >> 2);
                c.alive = true;
                c.leaf = true;
                c.parent = op.slot;
                c.morton = morton_encode(shadow_[c.inst], c.level, c.bx, c.by, c.bz);
                map_[key(c.inst, c.level, c.bx, c.by, c.bz)] = s;
                ++n_alive_;
                p.child[o] = s;
            }
            p.leaf = false;
        }
    }
}

std::vector<int> Topology::alive_sorted() const {
    std::vector<int> v;
    v.reserve(n_alive_);
    for (int s = 0; s < (int)blocks_.size(); ++s)
        if (blocks_[s].alive) v.push_back(s);
    std::sort(v.begin(), v.end(), [&](int a, int b) {
        const HostBlock &A = blocks_[a], &B = blocks_[b];
        if (A.inst != B.inst) return A.inst < B.inst;
        if (A.level != B.level) return A.level < B.level;
        return A.morton < B.morton;
    });
    return v;
}

void Topology::build(std::vector<BlockMeta> &meta, std::vector<int32_t> &child,
                     std::vector<int32_t> &nbr, HostLists &L) const {
    const int cap = capacity();
    meta.assign(cap, BlockMeta{0, 0, 0, 0, 0, -1, 0, 0, 0, -1, 0});
    child.assign((size_t)cap * 8, -1);
    nbr.assign((size_t)cap * 27, -2);
    const std::vector<int> order = alive_sorted();
    int maxl = 0;
    for (int s : order) maxl = std::max(maxl, blocks_[s].level);
    for (int s : order) {
        const HostBlock &b = blocks_[s];
        const mrfv_instance &p = inst_[b.inst];
        BlockMeta m{b.inst, b.level, b.bx, b.by, b.bz, b.parent, b.leaf ? 1 : 0, 0, 0, -1, 0};
        const int c[3] = {b.bx, b.by, b.bz};
        for (int a = 0; a < 3; ++a) {
            const int n = p.n0[a] << b.level;
            if (p.bc[a] != MRFV_BC_PERIODIC) {
                // boundary bit, plus bit 6 + side (mirror) or 12 + side (fixed values)
                const int mir = p.bc[a] == MRFV_BC_SYMMETRY ? 65 : (p.bc[a] == MRFV_BC_FIXED ? 4097 : 1);
                if (c[a] == 0) m.zg |= mir << (2 * a);
                if (c[a] == n - 1) m.zg |= mir << (2 * a + 1);
            }
        }
        meta[s] = m;
        for (int o = 0; o < 8; ++o) child[(size_t)s * 8 + o] = b.child[o];
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int d[3] = {dx, dy, dz};
                    int q[3];
                    bool outside = false;
                    for (int a = 0; a < 3; ++a) {
                        const int n = p.n0[a] << b.level;
                        int v = c[a] + d[a];
                        if (v < 0 || v >= n) {
                            if (p.bc[a] != MRFV_BC_PERIODIC) outside = true;
                            v = (v + n) % n;
                        }
                        q[a] = v;
                    }
                    const int idx = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                    nbr[(size_t)s * 27 + idx] =
                        outside ? -2 : find(b.inst, b.level, q[0], q[1], q[2]);
                }
    }
    // leaves whose stage result is final after the fused kernel (no jump correction of
    // their boundary cells) restrict themselves into their parent
    for (int s : order) {
        const HostBlock &b = blocks_[s];
        if (!b.leaf || b.parent < 0) continue;
        bool coarse_side = false;
        for (int r : {12, 14, 10, 16, 4, 22}) {
            const int nb = nbr[(size_t)s * 27 + r];
            if (nb >= 0 && !blocks_[nb].leaf) coarse_side = true;
        }
        meta[s].srestr = coarse_side ? 0 : 1;
    }
    // Halo regions of the prediction sources that a stage's predictions read.  A region of
    // block s (direction r) is predicted from the parent when, with the axes that point at
    // a clamped boundary taken out, it has no same-level neighbour (and no fixed values).
    // Its cells, and the evaluation points of clamped axes, lie along axis a within the
    // parent's cells (octant o): r_a = 0 -> the interior and the halo on side o_a (two
    // layers); r_a pointing out of the parent -> that side's halo and the interior; r_a
    // pointing at the sibling -> the interior only (the five-point stencils included).
    // Leaves mark their parents for the predicted face regions of a stage's fill, then
    // masked regions that are predicted themselves mark the next coarser level.
    auto predicted = [&](int s, int reg) {
        const int32_t zg = meta[s].zg;
        const int r[3] = {reg % 3 - 1, (reg / 3) % 3 - 1, reg / 9 - 1};
        int q[3];
        for (int a = 0; a < 3; ++a) {
            const int side = r[a] < 0 ? 0 : 1;
            if (r[a] != 0 && ((zg >> (12 + 2 * a + side)) & 1)) return false;   // fixed values
            q[a] = (r[a] != 0 && ((zg >> (2 * a + side)) & 1)) ? 0 : r[a];
        }
        if (q[0] == 0 && q[1] == 0 && q[2] == 0) return false;   // own cells (clamped)
        return nbr[(size_t)s * 27 + (q[2] + 1) * 9 + (q[1] + 1) * 3 + (q[0] + 1)] < 0;
    };
    auto need = [&](int s, int reg) {
        const HostBlock &b = blocks_[s];
        const int o[3] = {b.bx & 1, b.by & 1, b.bz & 1};
        const int r[3] = {reg % 3 - 1, (reg / 3) % 3 - 1, reg / 9 - 1};
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            const int d = r[a] == 0 ? (o[a] ? 1 : -1) : ((r[a] > 0) == (o[a] == 1) ? r[a] : 0);
            lo[a] = std::min(0, d);
            hi[a] = std::max(0, d);
        }
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) {
                    const int g = (z + 1) * 9 + (y + 1) * 3 + (x + 1);
                    if (g != 13) meta[b.parent].pmask |= 1 << (g < 13 ? g : g - 1);
                }
    };
    for (int s : order)
        if (blocks_[s].leaf && blocks_[s].parent >= 0)
            for (int reg : {12, 14, 10, 16, 4, 22})
                if (predicted(s, reg)) need(s, reg);
    for (int l = maxl; l >= 1; --l)
        for (int s : order)
            if (blocks_[s].level == l && !blocks_[s].leaf && meta[s].pmask)
                for (int i = 0; i < 26; ++i) {
                    const int reg = i < 13 ? i : i + 1;
                    if (((meta[s].pmask >> i) & 1) && predicted(s, reg)) need(s, reg);
                }
    // work lists
    const int n_inst = (int)inst_.size();
    L.data.assign(2 * n_inst, 0);
    L.max_level = maxl;
    L.lvl_off.assign(maxl + 1, 0);
    L.lvl_cnt.assign(maxl + 1, 0);
    L.par_off.assign(maxl + 1, 0);
    L.par_cnt.assign(maxl + 1, 0);
    L.leaf_off.assign(maxl + 1, 0);
    L.leaf_cnt.assign(maxl + 1, 0);
    L.jleaf_off.assign(maxl + 1, 0);
    L.jleaf_cnt.assign(maxl + 1, 0);
    L.j26_off.assign(maxl + 1, 0);
    L.j26_cnt.assign(maxl + 1, 0);
    L.pfill_off.assign(maxl + 1, 0);
    L.pfill_cnt.assign(maxl + 1, 0);
    L.pproj_off.assign(maxl + 1, 0);
    L.pproj_cnt.assign(maxl + 1, 0);
    L.par_srestr.assign(maxl + 1, 0);
    L.pproj_srestr.assign(maxl + 1, 0);
    auto all_srestr = [&](int off, int cnt) {
        for (int t = off; t < off + cnt; ++t)
            for (int o = 0; o < 8; ++o) {
                const int c = blocks_[L.data[t]].child[o];
                if (c < 0 || !meta[c].srestr) return false;
            }
        return true;
    };
    // prediction sources of a stage, marked fine to coarse
    std::vector<char> pf(cap, 0);
    auto lacks = [&](int s, bool faces_only) {
        const BlockMeta &m = meta[s];
        for (int r = 0; r < 27; ++r) {
            if (r == 13) continue;
            const int rx = r % 3 - 1, ry = (r / 3) % 3 - 1, rz = r / 9 - 1;
            if (faces_only && (rx != 0) + (ry != 0) + (rz != 0) != 1) continue;
            const bool zg = (rx < 0 && (m.zg & 1)) || (rx > 0 && (m.zg & 2)) || (ry < 0 && (m.zg & 4)) ||
                            (ry > 0 && (m.zg & 8)) || (rz < 0 && (m.zg & 16)) || (rz > 0 && (m.zg & 32));
            if (!zg && nbr[(size_t)s * 27 + r] < 0) return true;
        }
        return false;
    };
    for (int s : order)
        if (blocks_[s].leaf && blocks_[s].parent >= 0 && lacks(s, true)) pf[blocks_[s].parent] = 1;
    for (int l = maxl; l >= 1; --l)
        for (int s : order)
            if (blocks_[s].level == l && pf[s] && lacks(s, false) && blocks_[s].parent >= 0)
                pf[blocks_[s].parent] = 1;
    // interiors a stage reads, then their non-leaf descendants (restricted bottom-up first)
    std::vector<char> pr(cap, 0);
    auto mark_nonleaf = [&](int nb) {
        if (nb >= 0 && !blocks_[nb].leaf) pr[nb] = 1;
    };
    for (int s : order) {
        const HostBlock &b = blocks_[s];
        if (pf[s]) {
            pr[s] = 1;
            for (int r = 0; r < 27; ++r)
                if (r != 13) mark_nonleaf(nbr[(size_t)s * 27 + r]);
        }
        if (b.leaf)
            for (int r : {12, 14, 10, 16, 4, 22}) mark_nonleaf(nbr[(size_t)s * 27 + r]);   // faces
    }
    for (int l = 0; l <= maxl; ++l)
        for (int s : order)
            if (blocks_[s].level == l && pr[s])
                for (int o = 0; o < 8; ++o) mark_nonleaf(blocks_[s].child[o]);
    const int face_region[6] = {12, 14, 10, 16, 4, 22};
    auto needs_face_fill = [&](int s) {
        const BlockMeta &m = meta[s];
        for (int f = 0; f < 6; ++f)
            if ((m.zg >> f) & 1 || nbr[(size_t)s * 27 + face_region[f]] < 0) return true;
        return false;
    };
    auto needs_region_fill = [&](int s) {
        const BlockMeta &m = meta[s];
        if (m.zg) return true;
        for (int r = 0; r < 27; ++r)
            if (r != 13 && nbr[(size_t)s * 27 + r] < 0) return true;
        return false;
    };
    for (int l = 0; l <= maxl; ++l) {
        L.lvl_off[l] = (int32_t)L.data.size();
        for (int s : order)
            if (blocks_[s].level == l) L.data.push_back(s);
        L.lvl_cnt[l] = (int32_t)L.data.size() - L.lvl_off[l];
        L.par_off[l] = (int32_t)L.data.size();
        for (int s : order)
            if (blocks_[s].level == l && !blocks_[s].leaf) L.data.push_back(s);
        L.par_cnt[l] = (int32_t)L.data.size() - L.par_off[l];
        L.leaf_off[l] = (int32_t)L.data.size();
        for (int s : order)
            if (blocks_[s].level == l && blocks_[s].leaf) L.data.push_back(s);
        L.leaf_cnt[l] = (int32_t)L.data.size() - L.leaf_off[l];
        L.jleaf_off[l] = (int32_t)L.data.size();
        for (int s : order)
            if (blocks_[s].level == l && blocks_[s].leaf && needs_face_fill(s)) L.data.push_back(s);
        L.jleaf_cnt[l] = (int32_t)L.data.size() - L.jleaf_off[l];
        for (int t = L.jleaf_off[l]; t < L.jleaf_off[l] + L.jleaf_cnt[l] && !L.parents_needed; ++t) {
            const int sl = L.data[t];
            for (int f = 0; f < 6; ++f)
                if (!((meta[sl].zg >> f) & 1) && nbr[(size_t)sl * 27 + face_region[f]] < 0) L.parents_needed = true;
        }
        for (int s : order) {
            if (blocks_[s].level != l || !blocks_[s].leaf || L.parents_needed) continue;
            for (int f = 0; f < 6; ++f) {
                const int nb = nbr[(size_t)s * 27 + face_region[f]];
                if (nb >= 0 && !blocks_[nb].leaf) L.parents_needed = true;
            }
        }
        L.j26_off[l] = (int32_t)L.data.size();
        for (int s : order)
            if (blocks_[s].level == l && blocks_[s].leaf && needs_region_fill(s)) L.data.push_back(s);
        L.j26_cnt[l] = (int32_t)L.data.size() - L.j26_off[l];
        L.pfill_off[l] = (int32_t)L.data.size();
        for (int s : order)
            if (blocks_[s].level == l && !blocks_[s].leaf && pf[s] && meta[s].pmask) L.data.push_back(s);
        L.pfill_cnt[l] = (int32_t)L.data.size() - L.pfill_off[l];
        L.pproj_off[l] = (int32_t)L.data.size();
        for (int s : order)
            if (blocks_[s].level == l && !blocks_[s].leaf && pr[s]) L.data.push_back(s);
        L.pproj_cnt[l] = (int32_t)L.data.size() - L.pproj_off[l];
        L.par_srestr[l] = all_srestr(L.par_off[l], L.par_cnt[l]);
        L.pproj_srestr[l] = all_srestr(L.pproj_off[l], L.pproj_cnt[l]);
    }
    L.all_leaves_off = (int32_t)L.data.size();
    for (int i = 0; i < n_inst; ++i) {
        L.data[i] = (int32_t)L.data.size();
        for (int s : order)
            if (blocks_[s].leaf && blocks_[s].inst == i) L.data.push_back(s);
        L.data[n_inst + i] = (int32_t)L.data.size() - L.data[i];
    }
    L.all_leaves_cnt = (int32_t)L.data.size() - L.all_leaves_off;
    for (int t = 0; t < L.all_leaves_cnt; ++t) meta[L.data[L.all_leaves_off + t]].lpos = t;
    L.all_blocks_off = (int32_t)L.data.size();
    for (int s : order) L.data.push_back(s);
    L.all_blocks_cnt = (int32_t)L.data.size() - L.all_blocks_off;
    L.fine_off = (int32_t)L.data.size();
    for (int s : order)
        if (blocks_[s].level >= 1) L.data.push_back(s);
    L.fine_cnt = (int32_t)L.data.size() - L.fine_off;
    L.jcorr_off = (int32_t)L.data.size();
    for (int s : order) {
        if (!blocks_[s].leaf) continue;
        bool coarse_side = false;
        for (int r : {12, 14, 10, 16, 4, 22}) {
            const int nb = nbr[(size_t)s * 27 + r];
            if (nb >= 0 && !blocks_[nb].leaf) coarse_side = true;
        }
        if (coarse_side) L.data.push_back(s);
    }
    L.jcorr_cnt = (int32_t)L.data.size() - L.jcorr_off;
    L.pars_off = (int32_t)L.data.size();
    L.pars_copy_only = true;
    for (int s : order)
        if (!blocks_[s].leaf) {
            L.data.push_back(s);
            if (blocks_[s].level >= 1 && needs_region_fill(s)) L.pars_copy_only = false;
        }
    L.pars_cnt = (int32_t)L.data.size() - L.pars_off;
    L.desc.assign(2 * N_DESC, 0);
    auto set = [&](int which, int32_t off, int32_t cnt) {
        L.desc[2 * which] = off;
        L.desc[2 * which + 1] = cnt;
    };
    set(DESC_LEAVES, L.all_leaves_off, L.all_leaves_cnt);
    set(DESC_ALL, L.all_blocks_off, L.all_blocks_cnt);
    set(DESC_FINE, L.fine_off, L.fine_cnt);
    set(DESC_JCORR, L.jcorr_off, L.jcorr_cnt);
    set(DESC_PARS, L.pars_off, L.pars_cnt);
    for (int l = 0; l <= maxl && l < MAX_LEVELS; ++l) {
        set(desc_lvl(l), L.lvl_off[l], L.lvl_cnt[l]);
        set(desc_par(l), L.par_off[l], L.par_cnt[l]);
        set(desc_leaf(l), L.leaf_off[l], L.leaf_cnt[l]);
        set(desc_jleaf(l), L.jleaf_off[l], L.jleaf_cnt[l]);
        set(desc_jleaf26(l), L.j26_off[l], L.j26_cnt[l]);
        set(desc_pfill(l), L.pfill_off[l], L.pfill_cnt[l]);
        set(desc_pproj(l), L.pproj_off[l], L.pproj_cnt[l]);
    }
}

}  // namespace mrfv

extern "C" uint64_t mrfv_morton_encode(int32_t shadow, int32_t level, int32_t bx, int32_t by,
                                       int32_t bz) {
    return mrfv::morton_encode(shadow, level, bx, by, bz);
}

extern "C" uint64_t mrfv_morton_neighbor(uint64_t id, int32_t shadow, int32_t d, int32_t dir,
                                         int32_t *wrapped) {
    // decode -> shift one block along axis d -> encode (periodic image at the edge)
    int msb = 63;
    while (msb > 0 && !((id >> msb) & 1ull)) --msb;
    const int groups = msb / 3;
    const uint64_t body = id & ((1ull << (3 * groups)) - 1);
    int c[3] = {(int)mrfv::compact3(body), (int)mrfv::compact3(body >> 1),
                (int)mrfv::compact3(body >> 2)};
    const int n = 1 << groups;
    c[d] += dir;
    int w = 0;
    if (c[d] < 0 || c[d] >= n) {
        w = 1;
        c[d] = (c[d] + n) % n;
    }
    if (wrapped) *wrapped = w;
    return mrfv::morton_encode(shadow, groups - shadow, c[0], c[1], c[2]);
}
