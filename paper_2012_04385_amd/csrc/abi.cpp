// abi.cpp -- C ABI of the library: context, tree bookkeeping and the order of kernel
// launches for initialisation (algo:Init) and the global time step (algo:ComputeLoop).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mrfv_internal.h"

using namespace mrfv;

namespace {

int fail(mrfv_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

#define HIP_OK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(ctx, MRFV_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define CALL(expr)                                                                         \
    do {                                                                                   \
        int r_ = (expr);                                                                   \
        if (r_ != MRFV_OK) return r_;                                                      \
    } while (0)

size_t elem_size(const mrfv_ctx *ctx) { return ctx->cfg.dtype == MRFV_F64 ? 8 : 4; }

int check_instance(mrfv_ctx *ctx, const mrfv_instance &p, int i) {
    const std::string w = "instance " + std::to_string(i) + ": ";
    if (!(p.gamma > 1.0)) return fail(ctx, MRFV_EINVAL, w + "gamma must be > 1");
    if (!(p.dx0 > 0.0)) return fail(ctx, MRFV_EINVAL, w + "dx0 must be > 0");
    if (!(p.cfl > 0.0)) return fail(ctx, MRFV_EINVAL, w + "cfl must be > 0");
    if (!(p.eps >= 0.0)) return fail(ctx, MRFV_EINVAL, w + "eps must be >= 0");
    if (!(p.scale_rho > 0.0) || !(p.scale_E > 0.0))
        return fail(ctx, MRFV_EINVAL, w + "detail scales must be > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p.gravity[a])) return fail(ctx, MRFV_EINVAL, w + "gravity must be finite");
    if (p.lmax < 0 || p.lmax > 12) return fail(ctx, MRFV_EINVAL, w + "lmax must be in [0,12]");
    if (!(p.mu >= 0.0) || !std::isfinite(p.mu)) return fail(ctx, MRFV_EINVAL, w + "mu must be finite and >= 0");
    if (p.eos != MRFV_STIFFENED_GAS && p.eos != MRFV_TAIT)
        return fail(ctx, MRFV_EINVAL, w + "eos must be 0 (stiffened gas) or 1 (Tait)");
    if (p.eos == MRFV_TAIT) {
        if (!(p.B > 0.0) || !(p.tait_rho0 > 0.0) || !std::isfinite(p.tait_A))
            return fail(ctx, MRFV_EINVAL, w + "Tait needs B > 0, rho0 > 0 and a finite A");
        if (p.gravity[0] != 0.0 || p.gravity[1] != 0.0 || p.gravity[2] != 0.0)
            return fail(ctx, MRFV_EINVAL, w + "Tait has no energy equation for the gravity source");
    }
    for (int a = 0; a < 3; ++a) {
        if (p.n0[a] < 1 || ((int64_t)p.n0[a] << p.lmax) > 65535)
            return fail(ctx, MRFV_EINVAL, w + "n0 out of range");
        if (p.bc[a] < MRFV_BC_PERIODIC || p.bc[a] > MRFV_BC_FIXED)
            return fail(ctx, MRFV_EINVAL, w + "bc must be 0, 1, 2 or 3");
        if (p.bc[a] == MRFV_BC_FIXED) {
            if (!p.bc_fixed) return fail(ctx, MRFV_EINVAL, w + "fixed-value boundary without bc_fixed");
            for (int sd = 0; sd < 2; ++sd)
                for (int n = 0; n < (p.lmax + 1) * 4; ++n) {
                    const double *v = p.bc_fixed + ((size_t)(2 * a + sd) * (p.lmax + 1) * 4 + n) * 5;
                    bool ok = v[0] > 0.0 && (p.eos == MRFV_TAIT || v[4] + p.B > 0.0);
                    for (int q = 0; q < 5; ++q) ok = ok && std::isfinite(v[q]);
                    if (!ok) return fail(ctx, MRFV_EINVAL, w + "bc_fixed: needs finite states with rho > 0, p + B > 0");
                }
        }
    }
    return MRFV_OK;
}

// Flux kernel of the context's leaves: the configured scheme, or the Tait system's kernel.
int flux_kernel(const mrfv_ctx *ctx) { return ctx->inst[0].eos == MRFV_TAIT ? 4 : ctx->cfg.scheme; }

// A jump face exists when some leaf has a non-leaf same-level face neighbour.
bool any_jump(const Topology &tp, const HostLists &L, const std::vector<int32_t> &nbr) {
    const int faces[6] = {12, 14, 10, 16, 4, 22};
    for (int t = 0; t < L.all_leaves_cnt; ++t) {
        const int s = L.data[L.all_leaves_off + t];
        for (int f = 0; f < 6; ++f) {
            const int nb = nbr[(size_t)s * 27 + faces[f]];
            if (nb >= 0 && !tp.block(nb).leaf) return true;
        }
    }
    return false;
}

// Rebuild the device tables from the host tree.
int upload_tables(mrfv_ctx *ctx) {
    std::vector<BlockMeta> meta;
    std::vector<int32_t> child, nbr;
    ctx->topo.build(meta, child, nbr, ctx->lists);
    if ((int)ctx->lists.data.size() > ctx->lists_cap)
        return fail(ctx, MRFV_ENOMEM, "work-list capacity exceeded");
    hipStream_t st = ctx->stream;
    HIP_OK(hipMemcpyAsync(ctx->tb.meta, meta.data(), meta.size() * sizeof(BlockMeta),
                          hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->tb.child, child.data(), child.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->tb.nbr, nbr.data(), nbr.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->tb.lists, ctx->lists.data.data(),
                          ctx->lists.data.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->d_desc, ctx->lists.desc.data(), ctx->lists.desc.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));   // host vectors die at return
    ctx->has_jumps = any_jump(ctx->topo, ctx->lists, nbr);
    return MRFV_OK;
}

// Work lists.  Eager: offset and count from the host tree, one workgroup per block.
// Captured (ctx->capturing): offset and count read on the device from the descriptor
// table, grid bounded by the capacity, so the graph stays valid when the tree changes
// as long as the same lists are empty (the graph's key, graph_key); lists empty at
// capture are left out of the graph.
WorkList wlist(const mrfv_ctx *ctx, int which, int grid_cap = 2048, bool gated = true) {
    WorkList w;
    w.base = ctx->tb.lists;
    if (ctx->capturing) {
        // as gated by the graph's CFL reduction (see do_stages), or as uploaded
        w.desc = (gated ? ctx->d_desc_g : ctx->d_desc) + 2 * which;
        const std::vector<int32_t> &d = ctx->lists.desc;
        if (2 * which + 1 >= (int)d.size() || d[2 * which + 1] == 0) return w;   // grid 0: skipped
        // bound: the most blocks the list can ever hold (per level: every instance full)
        int64_t bound = ctx->cfg.slot_capacity;
        if (which >= desc_lvl(0) && which < desc_lvl(0) + DESC_PER_LEVEL * MAX_LEVELS)   // per-level lists
            bound = std::min<int64_t>(bound, ctx->lvl_bound[(which - desc_lvl(0)) / DESC_PER_LEVEL]);
        w.grid = (int)std::min<int64_t>(bound, grid_cap);
    } else {
        const std::vector<int32_t> &d = ctx->lists.desc;
        if (2 * which + 1 < (int)d.size()) {
            w.off = d[2 * which];
            w.n = d[2 * which + 1];
        }
        w.grid = w.n;
    }
    return w;
}

// Deepest level whose lists a launch sequence must cover.
int levels_to_cover(const mrfv_ctx *ctx) {
    return ctx->lists.max_level;
}

// stage_only: restrict only the parents a fused stage reads (desc_pproj), else all.
// skip_srestr: octants of children with meta.srestr hold the restriction the last fused
// stage wrote and are not recomputed.
template <typename T>
int do_project(mrfv_ctx *ctx, T *U, bool stage_only = false, bool rho_e_only = false,
               bool skip_srestr = false) {
    const HostLists &L = ctx->lists;
    for (int l = levels_to_cover(ctx) - 1; l >= 0; --l) {
        // a pass that skips the srestr octants has nothing to do when every child is one
        if (skip_srestr && (stage_only ? L.pproj_srestr[l] : L.par_srestr[l])) continue;
        HIP_OK(launch_project<T>(U, wlist(ctx, stage_only ? desc_pproj(l) : desc_par(l)), ctx->tb,
                                 ctx->stream, rho_e_only ? 0x11 : 0x1f, skip_srestr));
    }
    return MRFV_OK;
}

// Halo fill, levels coarse to fine (a prediction reads the parent's filled halo).
// Non-leaf blocks always get all 26 regions (they are prediction sources); leaves get
//   FILL_ALL: all 26 regions (explicit fill, refinement);
//   FILL_FACES: the face layers the flux reads (plain stages);
//   FILL_MISSING_FACES: faces without a same-level neighbour (fused stages, which read
//   same-level neighbours in place);
//   FILL_MISSING: all regions without a same-level neighbour (before the details, which
//   read same-level neighbours in place too).
// with_parents = false leaves the non-leaf blocks out (a stage on a tree where no leaf face
// reads a parent-derived value).
// FILL_RHO_E (with FILL_MISSING, before the details) applies to the parents' fill too.
template <typename T>
int do_fill(mrfv_ctx *ctx, T *U, int max_level, int mode = FILL_ALL, bool with_parents = true) {
    const int qsel = mode & FILL_RHO_E, m = mode & ~FILL_RHO_E;
    // before the details every non-leaf block gets its full halo; when that is copies only
    // (no prediction reads a coarser level's fill) one launch covers all levels
    const bool merged = m == FILL_MISSING && with_parents && ctx->lists.pars_copy_only &&
                        max_level >= levels_to_cover(ctx);
    if (merged)
        HIP_OK(launch_fill_halos<T>(U, wlist(ctx, DESC_PARS, 1024), ctx->tb, (FillMode)(FILL_ALL | qsel),
                                    ctx->stream));
    for (int l = 0; l <= std::min(max_level, levels_to_cover(ctx)); ++l) {
        if (m == FILL_ALL) {
            HIP_OK(launch_fill_halos<T>(U, wlist(ctx, desc_lvl(l), 1024), ctx->tb, (FillMode)mode,
                                        ctx->stream));
        } else {
            // a stage fills only the parents its predictions read; the fill before the
            // details (FILL_MISSING) all non-leaf blocks, whose details are judged too
            // (of those only the halo regions the predictions read)
            const int pw = m == FILL_MISSING_FACES ? desc_pfill(l) : desc_par(l);
            const int pm = m == FILL_MISSING_FACES ? FILL_MASKED : 0;
            if (with_parents && !merged)
                HIP_OK(launch_fill_halos<T>(U, wlist(ctx, pw, 1024), ctx->tb, (FillMode)(FILL_ALL | qsel | pm),
                                            ctx->stream));
            const int which = m == FILL_FACES ? desc_leaf(l)
                              : m == FILL_MISSING_FACES ? desc_jleaf(l) : desc_jleaf26(l);
            HIP_OK(launch_fill_halos<T>(U, wlist(ctx, which, 1024), ctx->tb, (FillMode)mode, ctx->stream));
        }
    }
    return MRFV_OK;
}

void timing_begin(mrfv_ctx *ctx, hipEvent_t *a) {
    if (!ctx->timing) return;
    if (ctx->ev_free.empty()) {
        hipEvent_t e;
        hipEventCreate(&e);
        ctx->ev_free.push_back(e);
    }
    *a = ctx->ev_free.back();
    ctx->ev_free.pop_back();
    hipEventRecord(*a, ctx->stream);
}

void timing_end(mrfv_ctx *ctx, hipEvent_t a, int64_t cells) {
    if (!ctx->timing) return;
    if (ctx->ev_free.empty()) {
        hipEvent_t e;
        hipEventCreate(&e);
        ctx->ev_free.push_back(e);
    }
    hipEvent_t b = ctx->ev_free.back();
    ctx->ev_free.pop_back();
    hipEventRecord(b, ctx->stream);
    ctx->ev_pairs.push_back(a);
    ctx->ev_pairs.push_back(b);
    ctx->ev_cells.push_back(cells);
}

// Flux differences D and boundary fluxes for all leaves, with the jump correction.
template <typename T>
int do_flux(mrfv_ctx *ctx, const T *U) {
    const HostLists &L = ctx->lists;
    if (!ctx->d_D) {   // the fused batched path never needs it; allocate on first use
        HIP_OK(hipStreamSynchronize(ctx->stream));
        if (hipMalloc(&ctx->d_D, (size_t)ctx->cfg.slot_capacity * 3 * 5 * CELLS_I * sizeof(T)) !=
            hipSuccess) {
            ctx->d_D = nullptr;
            return fail(ctx, MRFV_ENOMEM, "hipMalloc of the flux-difference scratch failed");
        }
    }
    T *D = (T *)ctx->d_D, *FF = (T *)ctx->d_FF;
    hipEvent_t ev{};
    timing_begin(ctx, &ev);
    if (ctx->cfg.batched) {
        HIP_OK(launch_flux<T>(flux_kernel(ctx), U, wlist(ctx, DESC_LEAVES), ctx->tb, ctx->d_inst, D, FF, ctx->stream));
    } else {
        for (int l = 0; l <= L.max_level; ++l)
            HIP_OK(launch_flux<T>(flux_kernel(ctx), U, wlist(ctx, desc_leaf(l)), ctx->tb, ctx->d_inst, D, FF,
                                  ctx->stream));
    }
    timing_end(ctx, ev, (int64_t)L.all_leaves_cnt * CELLS_I);
    // viscous terms: subtracted from the differences and face planes before the jump
    // correction averages the (total) fine fluxes
    if (ctx->viscous)
        HIP_OK(launch_visc<T>(U, wlist(ctx, DESC_LEAVES), ctx->tb, ctx->d_inst, D, FF, ctx->stream));
    if (ctx->has_jumps) {
        for (int l = L.max_level - 1; l >= 0; --l)
            HIP_OK(launch_ff_restrict<T>(FF, wlist(ctx, desc_par(l)), ctx->tb, ctx->stream));
        HIP_OK(launch_reflux<T>(D, FF, wlist(ctx, DESC_LEAVES), ctx->tb, ctx->stream));
    }
    return MRFV_OK;
}

// CFL time step of eq:Cfl per instance and, for viscous instances, the viscous bound.
template <typename T>
int do_cfl(mrfv_ctx *ctx, const T *U, double *dt) {
    const WorkList lv = wlist(ctx, DESC_LEAVES);
    HIP_OK(launch_cfl<T>(U, lv, ctx->tb, ctx->d_inst, (int)ctx->inst.size(), ctx->d_blockred, dt,
                         ctx->stream));
    if (ctx->viscous)
        HIP_OK(launch_visc_dt<T>(U, lv, ctx->tb, ctx->d_inst, (int)ctx->inst.size(), ctx->d_viscred, dt,
                                 ctx->stream));
    return MRFV_OK;
}

template <typename T>
int do_rhs(mrfv_ctx *ctx, const T *U, T *Lout) {
    CALL(do_flux<T>(ctx, U));
    const HostLists &L = ctx->lists;
    (void)L;
    HIP_OK(launch_combine<T>((const T *)ctx->d_D, Lout, wlist(ctx, DESC_LEAVES), ctx->tb,
                             ctx->d_inst, U, ctx->stream));
    return MRFV_OK;
}

template <typename T>
int do_update(mrfv_ctx *ctx, int stage, const double *dt, T *U, T *U0, const T *Lb) {
    HIP_OK(launch_update<T>(stage, dt, U, U0, Lb, wlist(ctx, DESC_LEAVES), ctx->tb, ctx->d_inst,
                            ctx->d_err, ctx->stream));
    return MRFV_OK;
}

// One stage of the batched path: fused rhs + update over all leaves, then the jump
// correction on the updated state.
int do_stage_fused(mrfv_ctx *ctx, int stage, const double *dt, const float *Uin, float *Uout,
                   float *U0, bool restrict_parents = false, double *cflmax = nullptr) {
    const HostLists &L = ctx->lists;
    float *FF = (float *)ctx->d_FF;
    hipEvent_t ev{};
    timing_begin(ctx, &ev);
    // the fused kernel has no grid-stride loop: its grid must cover every possible leaf
    HIP_OK(launch_rhs_update_f32(ctx->cfg.scheme, ctx->rhs_variant, stage, dt, Uin, Uout, U0, wlist(ctx, DESC_LEAVES, 1 << 30), ctx->tb,
                                 ctx->d_inst, FF, ctx->d_err, restrict_parents ? 1 : 0, cflmax, ctx->stream));
    timing_end(ctx, ev, (int64_t)L.all_leaves_cnt * CELLS_I);
    if (ctx->has_jumps) {
        for (int l = levels_to_cover(ctx) - 1; l >= 0; --l)
            HIP_OK(launch_ff_restrict<float>(FF, wlist(ctx, desc_par(l)), ctx->tb, ctx->stream));
        HIP_OK(launch_reflux_update<float>(stage, dt, Uout, FF, wlist(ctx, DESC_LEAVES), ctx->tb,
                                           ctx->d_inst, ctx->stream));
    }
    return MRFV_OK;
}

// flags_host / err_host (may be null): the flags and the error word are also written to
// host memory, read after the stream synchronises (no separate copies)
template <typename T>
int do_details_flags(mrfv_ctx *ctx, const T *U, int8_t *flags, double *det,
                     int8_t *flags_host = nullptr, int32_t *err_host = nullptr,
                     int32_t *gate = nullptr) {
    HIP_OK(launch_details<T>(U, wlist(ctx, DESC_FINE), ctx->tb, ctx->d_inst, ctx->d_det4, ctx->d_recheck, ctx->stream));
    HIP_OK(launch_flags(wlist(ctx, DESC_ALL), ctx->tb, ctx->d_inst, ctx->d_det4, det, flags, flags_host,
                        ctx->d_err, err_host, gate, ctx->cfg.slot_capacity, ctx->stream));
    return MRFV_OK;
}

// Device part of the adaptation up to the flags: the details read only rho and E, so
// parents are restricted and filled in those two (the fused path's last stage wrote the
// octants of jump-free leaves); all components are restricted and filled on the host's
// side when the flags change the tree.  gated: inside a step graph (the flags kernel
// records a tree change for the next launch's gate and writes the parity's half).
template <typename T>
int do_adapt_device(mrfv_ctx *ctx, T *U, bool gated) {
    const bool fused = ctx->cfg.batched && sizeof(T) == 4;
    CALL(do_project<T>(ctx, U, false, true, fused));
    CALL(do_fill<T>(ctx, U, 1 << 20, FILL_MISSING | FILL_RHO_E));
    CALL(do_details_flags<T>(ctx, U, ctx->d_flags, ctx->d_det, ctx->h_flags, ctx->h_err,
                             gated ? ctx->d_gate : nullptr));
    return MRFV_OK;
}

template <typename T>
int do_predict(mrfv_ctx *ctx, T *U, const int32_t *slots_host, int n, bool fill_parents = true) {
    if (n <= 0) return MRFV_OK;
    if (!fill_parents) {
        HIP_OK(hipMemcpyAsync(ctx->d_slots, slots_host, sizeof(int32_t) * n,
                              hipMemcpyHostToDevice, ctx->stream));
        HIP_OK(launch_predict<T>(U, ctx->d_slots, n, ctx->tb, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));   // slots_host may be a temporary
        return MRFV_OK;
    }
    // the parents' halos complete first: the prediction stencils reach 2 parent cells
    // beyond the child's octant, and a parent that was a leaf may have had only the
    // regions without a same-level neighbour filled
    std::vector<int32_t> par;
    for (int i = 0; i < n; ++i) {
        const int p = ctx->topo.block(slots_host[i]).parent;
        if (par.empty() || par.back() != p) par.push_back(p);
    }
    std::sort(par.begin(), par.end());
    par.erase(std::unique(par.begin(), par.end()), par.end());
    HIP_OK(hipMemcpyAsync(ctx->d_slots2, par.data(), sizeof(int32_t) * par.size(),
                          hipMemcpyHostToDevice, ctx->stream));
    WorkList wp;
    wp.base = ctx->d_slots2;
    wp.n = (int32_t)par.size();
    wp.grid = std::min<int>(wp.n, 1024);
    HIP_OK(launch_fill_halos<T>(U, wp, ctx->tb, FILL_ALL, ctx->stream));
    HIP_OK(hipMemcpyAsync(ctx->d_slots, slots_host, sizeof(int32_t) * n, hipMemcpyHostToDevice,
                          ctx->stream));
    HIP_OK(launch_predict<T>(U, ctx->d_slots, n, ctx->tb, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));   // slots_host may be a temporary
    return MRFV_OK;
}

int commit(mrfv_ctx *ctx, const int8_t *flags, std::vector<int32_t> &fresh) {
    std::vector<int> created;
    std::vector<TreeOp> ops;
    if (!ctx->topo.commit(flags, &ops, &created))
        return fail(ctx, MRFV_ENOMEM, "slot capacity exhausted");
    if (ops.empty()) return MRFV_OK;   // tree unchanged: the device tables stay valid
    fresh.insert(fresh.end(), created.begin(), created.end());
    return upload_tables(ctx);
}

// Turn per-leaf class scores into a committable proposal: refine only below l_max,
// coarsen only whole sibling groups of leaves on levels >= 2, nothing for non-adaptive
// instances.  mode 2 (persistence) proposes no change at all.
// net: the network's logits for this step are in h_logits (else the proposal is no change)
void decode_proposal(mrfv_ctx *ctx, const std::vector<int32_t> &leaves, bool net) {
    std::vector<int8_t> &P = ctx->proposal;
    P.assign(ctx->cfg.slot_capacity, 0);
    if (ctx->prop_mode != 1 || !net) return;
    const Topology &tp = ctx->topo;
    for (size_t r = 0; r < leaves.size(); ++r) {
        const float *z = ctx->h_logits + 3 * r;
        const int cls = (z[0] > z[1] && z[0] >= z[2]) ? 0 : (z[2] > z[1] ? 2 : 1);
        P[leaves[r]] = cls == 0 ? 1 : (cls == 2 ? -1 : 0);
    }
    for (int32_t s : leaves) {
        const HostBlock &b = tp.block(s);
        const mrfv_instance &I = ctx->inst[b.inst];
        if (!I.adapt) { P[s] = 0; continue; }
        if (P[s] == 1 && b.level >= I.lmax) P[s] = 0;
        if (P[s] == -1) {
            bool ok = b.level >= 2;
            if (ok) {
                const HostBlock &par = tp.block(b.parent);
                for (int o = 0; o < 8 && ok; ++o) {
                    const HostBlock &c = tp.block(par.child[o]);
                    ok = c.leaf && P[par.child[o]] == -1;
                }
            }
            if (!ok) P[s] = 0;
        }
    }
    // a group that lost a member above must drop the coarsen for every member
    for (int32_t s : leaves) {
        if (P[s] != -1) continue;
        const HostBlock &par = tp.block(tp.block(s).parent);
        for (int o = 0; o < 8; ++o)
            if (P[par.child[o]] != -1) { P[s] = 0; break; }
    }
}

// Commit the proposal on the host tree, build and stage its device tables on the side
// stream, then undo the commit.  Runs while the device computes the step.
int stage_proposal(mrfv_ctx *ctx) {
    HIP_OK(hipStreamSynchronize(ctx->side));   // last step's uploads still read s_*
    std::vector<TreeOp> ops;
    if (!ctx->topo.commit(ctx->proposal.data(), &ops, nullptr) || ops.empty()) {
        ctx->topo.undo(ops);
        ctx->staged = false;   // no change proposed, or it would not fit
        return MRFV_OK;
    }
    ctx->topo.build(ctx->s_meta, ctx->s_child, ctx->s_nbr, ctx->lists2);
    ctx->staged_jumps = any_jump(ctx->topo, ctx->lists2, ctx->s_nbr);
    ctx->topo.undo(ops);
    if ((int)ctx->lists2.data.size() > ctx->lists_cap) {
        ctx->staged = false;
        return MRFV_OK;
    }
    hipStream_t st = ctx->side;
    HIP_OK(hipMemcpyAsync(ctx->tb2.meta, ctx->s_meta.data(), ctx->s_meta.size() * sizeof(BlockMeta),
                          hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->tb2.child, ctx->s_child.data(), ctx->s_child.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->tb2.nbr, ctx->s_nbr.data(), ctx->s_nbr.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->tb2.lists, ctx->lists2.data.data(), ctx->lists2.data.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->d_desc2, ctx->lists2.desc.data(), ctx->lists2.desc.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, st));
    ctx->staged = true;
    return MRFV_OK;
}

// Adopt the staged tables after the judge confirmed the proposal: redo the same commit
// (the free list is in the same state, so the slots are the same) and copy the staged
// device tables over the live ones.
int adopt_staged(mrfv_ctx *ctx, std::vector<int32_t> &fresh) {
    std::vector<int> created;
    if (!ctx->topo.commit(ctx->proposal.data(), nullptr, &created))
        return fail(ctx, MRFV_ENOMEM, "slot capacity exhausted");
    fresh.insert(fresh.end(), created.begin(), created.end());
    HIP_OK(hipStreamSynchronize(ctx->side));
    hipStream_t st = ctx->stream;
    HIP_OK(hipMemcpyAsync(ctx->tb.meta, ctx->tb2.meta, ctx->s_meta.size() * sizeof(BlockMeta),
                          hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->tb.child, ctx->tb2.child, ctx->s_child.size() * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->tb.nbr, ctx->tb2.nbr, ctx->s_nbr.size() * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->tb.lists, ctx->tb2.lists, ctx->lists2.data.size() * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->d_desc, ctx->d_desc2, 2 * N_DESC * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    ctx->lists = ctx->lists2;
    ctx->has_jumps = ctx->staged_jumps;
    return MRFV_OK;
}

template <typename T>
int impose_ic(mrfv_ctx *ctx, mrfv_ic_fn ic, void *user, T *U, const std::vector<int> &slots) {
    std::vector<double> host((size_t)ctx->prim_batch * 5 * CELLS_I);
    for (size_t i0 = 0; i0 < slots.size(); i0 += ctx->prim_batch) {
        const int nb = (int)std::min<size_t>(ctx->prim_batch, slots.size() - i0);
        for (int k = 0; k < nb; ++k) {
            const HostBlock &b = ctx->topo.block(slots[i0 + k]);
            ic(user, b.inst, b.level, b.bx, b.by, b.bz, host.data() + (size_t)k * 5 * CELLS_I);
        }
        HIP_OK(hipMemcpyAsync(ctx->d_prim, host.data(), sizeof(double) * nb * 5 * CELLS_I,
                              hipMemcpyHostToDevice, ctx->stream));
        HIP_OK(hipMemcpyAsync(ctx->d_slots, slots.data() + i0, sizeof(int32_t) * nb,
                              hipMemcpyHostToDevice, ctx->stream));
        HIP_OK(launch_prim2cons<T>(ctx->d_prim, ctx->d_slots, nb, U, ctx->tb.meta, ctx->d_inst,
                                   ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
    }
    return MRFV_OK;
}

template <typename T>
int do_init(mrfv_ctx *ctx, mrfv_ic_fn ic, void *user, T *U) {
    Topology &tp = ctx->topo;
    tp.reset(ctx->cfg.slot_capacity, ctx->inst);
    std::vector<int> fresh;
    int maxl = 0;
    for (int i = 0; i < (int)ctx->inst.size(); ++i) {
        const mrfv_instance &p = ctx->inst[i];
        maxl = std::max(maxl, (int)p.lmax);
        for (int z = 0; z < p.n0[2]; ++z)
            for (int y = 0; y < p.n0[1]; ++y)
                for (int x = 0; x < p.n0[0]; ++x) {
                    const int s = tp.add_block(i, 0, x, y, z);
                    if (s < 0) return fail(ctx, MRFV_ENOMEM, "slot capacity exhausted");
                    fresh.push_back(s);
                }
    }
    CALL(upload_tables(ctx));
    CALL(impose_ic<T>(ctx, ic, user, U, fresh));
    std::vector<double> det(ctx->cfg.slot_capacity), det4((size_t)ctx->cfg.slot_capacity * details_parts());
    for (int m = 1; m <= maxl; ++m) {
        std::vector<int> parents;
        for (int s : tp.alive_sorted()) {
            const HostBlock &b = tp.block(s);
            if (b.level == m - 1 && ctx->inst[b.inst].lmax >= m) parents.push_back(s);
        }
        fresh.clear();
        for (int p : parents)
            if (!tp.refine(p, &fresh)) return fail(ctx, MRFV_ENOMEM, "slot capacity exhausted");
        CALL(upload_tables(ctx));
        CALL(impose_ic<T>(ctx, ic, user, U, fresh));
        if (m > 1 && !fresh.empty()) {
            CALL(do_fill<T>(ctx, U, m));
            HIP_OK(hipMemcpyAsync(ctx->d_slots, fresh.data(), sizeof(int32_t) * fresh.size(),
                                  hipMemcpyHostToDevice, ctx->stream));
            WorkList wf;
            wf.base = ctx->d_slots;
            wf.n = (int32_t)fresh.size();
            wf.grid = wf.n;
            HIP_OK(launch_details<T>(U, wf, ctx->tb, ctx->d_inst, ctx->d_det4, ctx->d_recheck, ctx->stream));
            const int nz = details_parts();
            HIP_OK(hipMemcpyAsync(det4.data(), ctx->d_det4, sizeof(double) * det4.size(),
                                  hipMemcpyDeviceToHost, ctx->stream));
            HIP_OK(hipStreamSynchronize(ctx->stream));
            for (int f : fresh)
                det[f] = *std::max_element(det4.begin() + (size_t)f * nz, det4.begin() + (size_t)(f + 1) * nz);
            for (int p : parents) {
                const HostBlock &b = tp.block(p);
                const mrfv_instance &P = ctx->inst[b.inst];
                const double eps = std::ldexp(P.eps, -3 * (P.lmax - m));
                bool small = true;
                for (int o = 0; o < 8; ++o)
                    if (!(det[b.child[o]] < eps)) small = false;
                if (small) tp.coarsen(p);
            }
            CALL(upload_tables(ctx));
        }
    }
    CALL(do_project<T>(ctx, U));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    ctx->initialised = true;
    return MRFV_OK;
}

// CFL step and the three RK stages.
template <typename T>
int do_stages(mrfv_ctx *ctx, T *U, T *U0, T *Lb, double *dt) {
    if (ctx->capturing) {
        // a step graph: the CFL step reads the ungated leaf list, and its per-instance
        // reduction gates the lists of every later kernel (a speculative step whose tree
        // was changed meanwhile computes a time step that the relaunched step replaces).
        // After a step on the same tree the block maxima are already there: that step's last
        // stage (and, at jumps, a pass after the correction) wrote them from its new state
        // (leaf interiors do not change after that).
        WorkList lv = wlist(ctx, DESC_LEAVES, 2048, false);
        if (ctx->cfl_from_stage) lv.grid = 0;
        HIP_OK(launch_cfl<T>(U, lv, ctx->tb, ctx->d_inst, (int)ctx->inst.size(), ctx->d_blockred,
                             dt, ctx->stream, ctx->d_gate, ctx->d_desc, ctx->d_desc_g, N_DESC));
    } else {
        CALL(do_cfl<T>(ctx, U, dt));
    }
    if (ctx->cfg.batched && sizeof(T) == 4) {
        // fused stages, out of place through two more state buffers: U -> W -> W2 -> U;
        // parents are restricted and filled only if some leaf face reads them.  Stages
        // whose output is restricted next (W and W2 when stages read parents, U before
        // the details) write the restriction of jump-free leaves into their parents, so
        // those restriction passes recompute only the other octants.  U comes from the
        // caller, who may have written it: the first stage restricts in full, except in a
        // step graph after a step on the same tree (the last stage of an adaptive step
        // restricts, and nothing changes leaf interiors after it).
        float *buf[4] = {(float *)U, (float *)ctx->d_W, (float *)ctx->d_W2, (float *)U};
        const bool par = ctx->lists.parents_needed;
        bool adapt = false;
        for (const auto &p : ctx->inst) adapt = adapt || (p.adapt && p.lmax > 0);
        for (int s = 0; s < 3; ++s) {
            float *in = buf[s], *out = buf[s + 1];
            const bool skip = s > 0 || (ctx->capturing && ctx->restrict_from_stage);
            if (par) CALL(do_project<float>(ctx, in, true, false, skip));
            CALL(do_fill<float>(ctx, in, 1 << 20, FILL_MISSING_FACES, par));
            // a step graph's last stage writes the block maxima of the signal speeds for the
            // next step's CFL pass; the leaves whose boundary cells the jump correction then
            // changes get theirs again from the corrected state
            double *cflmax = ctx->capturing && s == 2 ? ctx->d_blockred : nullptr;
            CALL(do_stage_fused(ctx, s, dt, in, out, (float *)U0, s < 2 ? par : adapt, cflmax));
            if (cflmax && ctx->has_jumps)
                HIP_OK(launch_cfl_blocks<float>(out, wlist(ctx, DESC_JCORR), ctx->tb, ctx->d_inst,
                                                ctx->d_blockred, ctx->stream));
        }
        return MRFV_OK;
    }
    // the viscous fluxes read the edge halos too
    const int fill = ctx->viscous ? FILL_ALL : FILL_FACES;
    for (int s = 0; s < 3; ++s) {
        CALL(do_project<T>(ctx, U));
        CALL(do_fill<T>(ctx, U, 1 << 20, fill));
        CALL(do_rhs<T>(ctx, U, Lb));
        CALL(do_update<T>(ctx, s, dt, U, U0, Lb));
    }
    return MRFV_OK;
}

// hipGraph of a step (batched FP32 path, batched == 2): the CFL step with the gate, the
// three RK stages and, for adaptive contexts, the adaptation up to the flags.  The kernels
// read their work lists through the gated device descriptors, so one capture serves every
// later tree.  Captured on the library's own stream, launched on the caller's.
// Which launches a captured step graph contains: the finest level present, whether
// resolution jumps exist, and which per-level lists are non-empty.  Counts and list
// contents are read on the device, so one graph serves every tree with the same key.
GraphKey graph_key(const mrfv_ctx *ctx) {
    const HostLists &L = ctx->lists;
    uint64_t k = (uint64_t)L.max_level | ((uint64_t)ctx->has_jumps << 4) |
                 ((uint64_t)L.parents_needed << 63) | ((uint64_t)ctx->cfl_from_stage << 62) |
                 ((uint64_t)ctx->restrict_from_stage << 61) | ((uint64_t)L.pars_copy_only << 60);
    uint64_t k2 = 0;
    for (int l = 0; l <= L.max_level && l < MAX_LEVELS; ++l) {
        if (L.desc[2 * desc_par(l) + 1] > 0) k |= 1ull << (5 + l);
        if (L.desc[2 * desc_jleaf(l) + 1] > 0) k |= 1ull << (5 + MAX_LEVELS + l);
        if (L.desc[2 * desc_pfill(l) + 1] > 0) k |= 1ull << (5 + 2 * MAX_LEVELS + l);
        if (L.desc[2 * desc_pproj(l) + 1] > 0) k |= 1ull << (5 + 3 * MAX_LEVELS + l);
        if (L.desc[2 * desc_jleaf26(l) + 1] > 0) k2 |= 1ull << l;   // the adaptation's fill
        if (L.par_srestr[l]) k2 |= 1ull << (MAX_LEVELS + l);            // restriction passes
        if (L.pproj_srestr[l]) k2 |= 1ull << (2 * MAX_LEVELS + l);      // left out
    }
    return {k, k2};
}

void drop_graphs(mrfv_ctx *ctx) {
    for (auto &kv : ctx->graphs) hipGraphExecDestroy(kv.second);
    ctx->graphs.clear();
}

int run_step_graph(mrfv_ctx *ctx, float *U, float *U0, double *dt, bool adapt) {
    if (ctx->gU != U || ctx->gU0 != U0 || ctx->gdt != dt) drop_graphs(ctx);
    const GraphKey key = graph_key(ctx);
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        if (ctx->graphs.size() >= 32) drop_graphs(ctx);   // bound the cache
        ctx->graph = nullptr;
        if (!ctx->gstream) HIP_OK(hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking));
        HIP_OK(hipStreamSynchronize(ctx->stream));
        hipStream_t user = ctx->stream;
        ctx->stream = ctx->gstream;
        ctx->capturing = true;
        hipError_t e = hipStreamBeginCapture(ctx->gstream, hipStreamCaptureModeThreadLocal);
        int rc = MRFV_EHIP;
        if (e == hipSuccess) {
            rc = do_stages<float>(ctx, U, U0, nullptr, dt);
            if (rc == MRFV_OK && adapt) rc = do_adapt_device<float>(ctx, U, true);
        }
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(ctx->gstream, &g);
        ctx->capturing = false;
        ctx->stream = user;
        if (e != hipSuccess || e2 != hipSuccess || rc != MRFV_OK || !g)
            return fail(ctx, MRFV_EHIP, "step graph capture failed");
        hipError_t e3 = hipGraphInstantiate(&ctx->graph, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e3 != hipSuccess) {
            ctx->graph = nullptr;
            return fail(ctx, MRFV_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
        }
        ctx->gU = U;
        ctx->gU0 = U0;
        ctx->gdt = dt;
        it = ctx->graphs.emplace(key, ctx->graph).first;
        ctx->graph = nullptr;
    }
    HIP_OK(hipGraphLaunch(it->second, ctx->stream));
    ctx->graph_launches++;
    return MRFV_OK;
}

// Device part of a step: stages and, for adaptive contexts, the restriction, fills,
// details and flags.  The batched FP32 path replays all of it as one graph whose CFL
// reduction gates the work lists (see k_cfl_inst); *half receives the half of the host flag
// buffers the flags go to.
template <typename T>
int launch_step(mrfv_ctx *ctx, T *U, T *U0, T *Lb, double *dt, bool adapt, int *half) {
    if (ctx->cfg.batched == 2 && sizeof(T) == 4 && !ctx->timing) {
        CALL(run_step_graph(ctx, (float *)U, (float *)U0, dt, adapt));
        *half = (int)(ctx->graph_launches & 1);
        return MRFV_OK;
    }
    CALL(do_stages<T>(ctx, U, U0, Lb, dt));
    if (adapt) CALL(do_adapt_device<T>(ctx, U, false));
    *half = 0;
    return MRFV_OK;
}

// Host part of an adaptive step once its flags are in host memory (half `half`): the
// error word, then, when the flags change the tree, the full restriction and fills on
// the old tree, the commit and the prediction of the new children.  *changed: whether
// the tree changed.
template <typename T>
int finish_step(mrfv_ctx *ctx, T *U, int half, bool prop, const std::vector<int32_t> &leaves,
                bool *changed) {
    using clk = std::chrono::steady_clock;
    auto ms = [](clk::time_point a, clk::time_point b) {
        return std::chrono::duration<double, std::milli>(b - a).count();
    };
    const auto w1 = clk::now();
    const int8_t *hf = ctx->h_flags + (size_t)half * ctx->cfg.slot_capacity;
    ctx->last_half = half;
    if (ctx->h_err[half]) return fail(ctx, MRFV_ENONPHYS, "non-physical state (rho<=0, p+B<=0 or NaN)");
    bool change = false;
    {
        // The details saw rho and E only.  When the tree changes, on the old tree and
        // before it changes: every component is restricted (a coarsened parent becomes a
        // leaf with its restricted values), the parents' halos are filled, and then the
        // full halos of the leaves to be refined, whose children are predicted from them
        // (after the commit a same-level neighbour of such a leaf can be a fresh child
        // that holds no data yet).
        const HostLists &L = ctx->lists;
        std::vector<int32_t> refined;
        for (int i = 0; i < L.all_leaves_cnt; ++i) {
            const int32_t sl = L.data[L.all_leaves_off + i];
            const int8_t f = hf[sl];
            change = change || f == 1 || f == -1;
            if (f == 1) refined.push_back(sl);
        }
        if (change) {
            CALL(do_project<T>(ctx, U));
            CALL(do_fill<T>(ctx, U, 1 << 20, FILL_MISSING));
        }
        if (!refined.empty()) {
            HIP_OK(hipMemcpyAsync(ctx->d_slots2, refined.data(), sizeof(int32_t) * refined.size(),
                                  hipMemcpyHostToDevice, ctx->stream));
            WorkList wr;
            wr.base = ctx->d_slots2;
            wr.n = (int32_t)refined.size();
            wr.grid = std::min<int>(wr.n, 1024);
            HIP_OK(launch_fill_halos<T>(U, wr, ctx->tb, FILL_ALL, ctx->stream));
            // refined lives until the copy has been read
            HIP_OK(hipStreamSynchronize(ctx->stream));
        }
    }
    std::vector<int32_t> fresh;
    bool tree_changed = change;
    if (prop) {
        bool hit = true;
        for (int32_t s : leaves) {
            const int j = hf[s], q = ctx->proposal[s];
            const int cj = j == 1 ? 0 : (j == -1 ? 2 : 1), cq = q == 1 ? 0 : (q == -1 ? 2 : 1);
            if (j != q) hit = false;
            if (cj == cq) ctx->p_tp[cj]++;
            else { ctx->p_fn[cj]++; ctx->p_fp[cq]++; }
        }
        ctx->p_steps++;
        bool pchange = false;
        for (int32_t sl : leaves) pchange = pchange || ctx->proposal[sl] != 0;
        if (hit) ctx->p_hits++;
        if (ctx->staged) ctx->p_staged++;
        if (hit && !pchange) {
            // nothing to commit
        } else if (hit && ctx->staged) {
            ctx->p_adopted++;
            CALL(adopt_staged(ctx, fresh));
        } else {
            CALL(commit(ctx, hf, fresh));
        }
    } else if (change) {   // flags without a refine or coarsen leave the tree as it is
        CALL(commit(ctx, hf, fresh));
    }
    const auto w2 = clk::now();
    CALL(do_predict<T>(ctx, U, fresh.data(), (int)fresh.size(), false));
    const auto w3 = clk::now();
    ctx->h_commit_ms += ms(w1, w2);
    ctx->h_predict_ms += ms(w2, w3);
    ctx->h_steps++;
    *changed = tree_changed;
    return MRFV_OK;
}

bool adaptive(const mrfv_ctx *ctx) {
    bool adapt = false;
    for (const auto &p : ctx->inst) adapt = adapt || (p.adapt && p.lmax > 0);
    return adapt;
}

template <typename T>
int do_step(mrfv_ctx *ctx, T *U, T *U0, T *Lb, double *dt) {
    const bool adapt = adaptive(ctx);
    const bool prop = adapt && ctx->prop_mode != 0;
    std::vector<int32_t> leaves;
    if (prop) {
        const HostLists &L = ctx->lists;
        leaves.assign(L.data.begin() + L.all_leaves_off,
                      L.data.begin() + L.all_leaves_off + L.all_leaves_cnt);
    }
    // the network runs only after a step that changed the tree (and on the first step): after
    // a step without change the proposal is "no change", which is right whenever the tree
    // stays as it is, at no cost
    const bool net = prop && ctx->prop_mode == 1 && !leaves.empty() && ctx->p_net_due;
    if (net) {
        ctx->p_net_runs++;
        // proposal for this step's judge from the state at its start; it is queued
        // ahead of the stages, so the host can read it while the device continues
        HIP_OK(launch_features<T>(U, wlist(ctx, DESC_LEAVES), ctx->tb, ctx->d_inst, ctx->d_X,
                                  ctx->stream));
        CALL(mlp_forward_on(ctx->mlp, ctx->stream, ctx->d_X, (int)leaves.size(), ctx->d_logits));
        HIP_OK(hipMemcpyAsync(ctx->h_logits, ctx->d_logits, leaves.size() * 3 * sizeof(float),
                              hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipEventRecord(ctx->ev_prop, ctx->stream));
    }
    // this step is not speculative: no earlier change may gate it
    HIP_OK(hipMemsetAsync(ctx->d_gate, 0, sizeof(int32_t), ctx->stream));
    int half = 0;
    CALL(launch_step<T>(ctx, U, U0, Lb, dt, adapt, &half));
    if (!adapt) return MRFV_OK;
    if (prop) {
        // host-side tree work for the proposed flags, overlapped with the device
        if (net) HIP_OK(hipEventSynchronize(ctx->ev_prop));
        const auto t0 = std::chrono::steady_clock::now();
        decode_proposal(ctx, leaves, net);
        CALL(stage_proposal(ctx));
        ctx->p_build_ms +=
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    const auto w0 = std::chrono::steady_clock::now();
    HIP_OK(hipStreamSynchronize(ctx->stream));
    ctx->h_wait_ms +=
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
    bool changed = false;
    CALL(finish_step<T>(ctx, U, half, prop, leaves, &changed));
    ctx->p_net_due = changed;
    return MRFV_OK;
}

// n steps.  On the graph path of an adaptive context without a proposer, step k+1 is
// launched before the host has read step k's flags; if those flags change the tree, the
// gate at the start of step k+1 zeroes its work lists (it does nothing), and step k+1 is
// launched again after the commit.  Otherwise the device runs the steps back to back.
template <typename T>
int do_run(mrfv_ctx *ctx, T *U, T *U0, T *Lb, double *dt, int n, int64_t *cells) {
    const bool adapt = adaptive(ctx);
    const bool spec = adapt && ctx->prop_mode == 0 && ctx->cfg.batched == 2 && sizeof(T) == 4 &&
                      !ctx->timing;
    auto leaf_cells = [&]() { return (int64_t)ctx->lists.all_leaves_cnt * CELLS_I; };
    *cells = 0;
    if (!spec) {
        for (int k = 0; k < n; ++k) {
            *cells += leaf_cells();
            CALL(do_step<T>(ctx, U, U0, Lb, dt));
        }
        return MRFV_OK;
    }
    if (n <= 0) return MRFV_OK;
    const std::vector<int32_t> none;
    hipEvent_t ev[2];
    HIP_OK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    if (hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) {
        hipEventDestroy(ev[0]);
        return fail(ctx, MRFV_EHIP, "hipEventCreate failed");
    }
    int rc = MRFV_OK;
    int half[2] = {0, 0};
    int64_t step_cells[2] = {0, 0};
    // whether the last launch wrote the CFL block maxima of its new state on the current
    // tree (the first launch of a call never uses them: the caller owns U)
    // and whether it restricted its leaves into their parents (every launch here adapts)
    bool stage_maxima = false, stage_restricted = false;
    auto launch = [&](int k) {
        step_cells[k & 1] = leaf_cells();   // the tree this launch integrates
        ctx->cfl_from_stage = stage_maxima;
        ctx->restrict_from_stage = stage_restricted;
        int r = launch_step<T>(ctx, U, U0, Lb, dt, true, &half[k & 1]);
        ctx->cfl_from_stage = ctx->restrict_from_stage = false;
        stage_maxima = r == MRFV_OK;
        stage_restricted = r == MRFV_OK;
        if (r == MRFV_OK && hipEventRecord(ev[k & 1], ctx->stream) != hipSuccess)
            r = fail(ctx, MRFV_EHIP, "hipEventRecord failed");
        return r;
    };
    if (hipMemsetAsync(ctx->d_gate, 0, sizeof(int32_t), ctx->stream) != hipSuccess)
        rc = fail(ctx, MRFV_EHIP, "hipMemsetAsync failed");
    if (rc == MRFV_OK) rc = launch(0);
    for (int k = 0; k < n && rc == MRFV_OK; ++k) {
        if (k + 1 < n && (rc = launch(k + 1)) != MRFV_OK) break;   // speculative
        const auto w0 = std::chrono::steady_clock::now();
        if (hipEventSynchronize(ev[k & 1]) != hipSuccess) {
            rc = fail(ctx, MRFV_EHIP, "hipEventSynchronize failed");
            break;
        }
        ctx->h_wait_ms +=
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
        bool changed = false;
        *cells += step_cells[k & 1];
        if ((rc = finish_step<T>(ctx, U, half[k & 1], false, none, &changed)) != MRFV_OK) break;
        if (changed) stage_maxima = stage_restricted = false;   // new leaves; step k+1 (if queued) was void
        if (changed && k + 1 < n) {
            // the speculative step k+1 was gated (it changed nothing): run it on the new tree
            if (hipMemsetAsync(ctx->d_gate, 0, sizeof(int32_t), ctx->stream) != hipSuccess) {
                rc = fail(ctx, MRFV_EHIP, "hipMemsetAsync failed");
                break;
            }
            rc = launch(k + 1);
        }
    }
    hipStreamSynchronize(ctx->stream);   // nothing of this call stays in flight
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    return rc;
}

// ---------------------------------------------------------- local time stepping ----
// eq:LtsTimestep, algo:ComputeLoop, algo:Integration on the plain kernels.  A macro step
// is 2^lmax micro steps r of dt (the eq:Cfl step of level lmax); level l completes a step
// of its own dt_l = 2^(lmax - l) dt at micro step r when r + 1 is a multiple of
// 2^(lmax - l).  A level's first stage is evaluated at the micro step its step starts in;
// its stages are integrated at the micro step it ends in.  Halo cells of faces without a
// same-level neighbour hold their own state, set by prediction when every level is at
// the same time (the macro step's start) and integrated in between with the flux
// divergence predicted from the coarser level.  Every leaf sums its boundary face fluxes
// with the RK weights; at the end of its step a coarse leaf next to a refined same-level
// neighbour replaces its own sum by the fine average (the coarse cell adjustment).

int lts_lowest_ending(int lmax, int r) { return lmax + 1 - __builtin_popcount((unsigned)((r + 1) ^ r)); }

template <typename T>
int lts_buffers(mrfv_ctx *ctx) {
    if (ctx->d_Fp && ctx->d_D) return MRFV_OK;
    HIP_OK(hipStreamSynchronize(ctx->stream));
    const size_t cap = ctx->cfg.slot_capacity, es = sizeof(T);
    struct Want { void **p; size_t bytes; } want[] = {
        {&ctx->d_D, cap * 3 * 5 * CELLS_I * es},
        {&ctx->d_Fp, cap * 5 * CELLS_P * es},
        {&ctx->d_H0, cap * 6 * 5 * (size_t)lts_halo_slab() * es},
        {&ctx->d_ACC, cap * 6 * 5 * FACE * es}};
    for (auto &w : want) {
        if (*w.p) continue;
        if (hipMalloc(w.p, w.bytes) != hipSuccess) {
            *w.p = nullptr;
            return fail(ctx, MRFV_ENOMEM, "hipMalloc of the local time stepping buffers failed");
        }
    }
    // halo regions of F that no kernel writes are never read; cleared once for tidiness
    HIP_OK(hipMemsetAsync(ctx->d_Fp, 0, cap * 5 * CELLS_P * es, ctx->stream));
    return MRFV_OK;
}

template <typename T>
int do_lts_macro(mrfv_ctx *ctx, T *U, T *U0, T *Lb, double *dt, int64_t *cell_updates) {
    CALL(lts_buffers<T>(ctx));
    const HostLists &L = ctx->lists;
    const int lmax = ctx->inst[0].lmax, top = levels_to_cover(ctx);
    T *D = (T *)ctx->d_D, *FF = (T *)ctx->d_FF, *F = (T *)ctx->d_Fp, *H0 = (T *)ctx->d_H0,
      *ACC = (T *)ctx->d_ACC;
    const size_t cap = ctx->cfg.slot_capacity;
    // FP32 flux divergence from the fused stage kernel (not Tait's system, which it lacks),
    // in the context's launch shape
    const bool fused = sizeof(T) == 4 && flux_kernel(ctx) != 4;
    int64_t cells = 0;
    for (int l = 0; l <= top; ++l) cells += (int64_t)L.leaf_cnt[l] * ((int64_t)1 << l) * CELLS_I;
    if (cell_updates) *cell_updates = cells;
    HIP_OK(launch_cfl<T>(U, wlist(ctx, DESC_LEAVES), ctx->tb, ctx->d_inst, (int)ctx->inst.size(),
                         ctx->d_blockred, dt, ctx->stream));
    // every level at the same time: parents and all face halos from the state
    CALL(do_project<T>(ctx, U));
    CALL(do_fill<T>(ctx, U, 1 << 20, FILL_FACES));
    HIP_OK(hipMemsetAsync(ACC, 0, cap * 6 * 5 * FACE * sizeof(T), ctx->stream));
    for (int r = 0; r < (1 << lmax); ++r) {
        const int lo_end = lts_lowest_ending(lmax, r);
        const int lo_start = r == 0 ? 0 : lts_lowest_ending(lmax, r - 1);
        for (int st = 0; st < 3; ++st) {
            const int lo_rhs = st == 0 ? lo_start : lo_end;
            // flux divergence of the leaves being evaluated, after their copied halos; in
            // FP32 the fused stage kernel evaluates it (reading same-level neighbours in
            // place, so only boundary halos are filled) straight into F
            for (int l = lo_rhs; l <= top; ++l) {
                const WorkList w = wlist(ctx, desc_leaf(l));
                if (fused) {
                    // the boundary faces (nothing else) when some axis is not periodic
                    if (ctx->bounded)
                        HIP_OK(launch_fill_halos<T>(U, w, ctx->tb, (FillMode)(FILL_MISSING_FACES | FILL_PRESENT),
                                                    ctx->stream));
                    // (leaves without a non-leaf same-level face neighbour also write the
                    // restriction of their L into the parent's octant of F)
                    HIP_OK(launch_rhs_update_f32(ctx->cfg.scheme, ctx->rhs_variant, -1, dt, (const float *)U, (float *)F,
                                                 (float *)U0, wlist(ctx, desc_leaf(l), 1 << 30), ctx->tb,
                                                 ctx->d_inst, (float *)FF, ctx->d_err, 1, nullptr, ctx->stream));
                    continue;
                }
                HIP_OK(launch_fill_halos<T>(U, w, ctx->tb, (FillMode)(FILL_FACES | FILL_PRESENT), ctx->stream));
                HIP_OK(launch_flux<T>(flux_kernel(ctx), U, w, ctx->tb, ctx->d_inst, D, FF, ctx->stream));
                HIP_OK(launch_lts_combine<T>(D, F, w, ctx->tb, ctx->d_inst, U, ctx->stream));
            }
            // averaged into the parents (in FP32 the octants the fused kernel wrote are
            // skipped: every leaf below these parents was evaluated in this stage), predicted
            // into the jump halos
            for (int p = top - 1; p >= std::max(lo_rhs, 1) - 1; --p) {
                if (fused && L.par_srestr[p]) continue;   // every child wrote its octant
                HIP_OK(launch_project<T>(F, wlist(ctx, desc_par(p)), ctx->tb, ctx->stream, 31, fused));
            }
            CALL(do_fill<T>(ctx, F, 1 << 20, FILL_MISSING_FACES, true));
            // algo:Integration of the levels that end a step at r
            for (int l = lo_end; l <= top; ++l)
                HIP_OK(launch_lts_update<T>(st, dt, U, U0, H0, F, FF, ACC, wlist(ctx, desc_leaf(l)), ctx->tb,
                                            ctx->d_inst, ctx->d_err, ctx->stream));
            if (st == 2 && ctx->has_jumps) {
                for (int p = top - 1; p >= lo_end; --p)
                    HIP_OK(launch_ff_restrict<T>(ACC, wlist(ctx, desc_par(p)), ctx->tb, ctx->stream));
                for (int l = lo_end; l <= top; ++l)
                    HIP_OK(launch_lts_adjust<T>(U, ACC, wlist(ctx, desc_leaf(l)), ctx->tb, ctx->d_inst,
                                                ctx->stream));
            }
            if (st == 2)
                HIP_OK(launch_lts_zero<T>(ACC, wlist(ctx, DESC_LEAVES), ctx->tb, lo_end, ctx->stream));
            for (int p = top - 1; p >= std::max(lo_end, 1) - 1; --p)
                HIP_OK(launch_project<T>(U, wlist(ctx, desc_par(p)), ctx->tb, ctx->stream));
        }
    }
    return MRFV_OK;
}

template <typename T>
int do_step_lts(mrfv_ctx *ctx, T *U, T *U0, T *Lb, double *dt, int64_t *cell_updates) {
    CALL(do_lts_macro<T>(ctx, U, U0, Lb, dt, cell_updates));
    if (!adaptive(ctx)) return MRFV_OK;
    CALL(do_adapt_device<T>(ctx, U, false));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    bool changed = false;
    return finish_step<T>(ctx, U, 0, false, {}, &changed);
}

int need_init(mrfv_ctx *ctx) {
    if (!ctx) return MRFV_EINVAL;
    if (!ctx->initialised) return fail(ctx, MRFV_ESTATE, "mrfv_init_blocks has not run");
    return MRFV_OK;
}

}  // namespace

extern "C" {

int mrfv_create(mrfv_ctx **out, const mrfv_config *cfg, const mrfv_instance *inst,
                void *hip_stream) {
    if (!out || !cfg || !inst) return MRFV_EINVAL;
    *out = nullptr;
    mrfv_ctx *ctx = new mrfv_ctx();
    auto bail = [&](int code) {
        mrfv_destroy(ctx);
        return code;
    };
    ctx->cfg = *cfg;
    ctx->rhs_variant = rhs_default_variant(cfg->scheme);
    if (cfg->dtype != MRFV_F32 && cfg->dtype != MRFV_F64) return bail(MRFV_EINVAL);
    if (cfg->n_instances < 1 || cfg->n_instances > 4095) return bail(MRFV_EINVAL);
    if (cfg->slot_capacity < 1 || cfg->slot_capacity > (1 << 22)) return bail(MRFV_EINVAL);
    if (cfg->scheme < MRFV_ROE_WENO5 || cfg->scheme > MRFV_HLLC_WAO53) return bail(MRFV_EINVAL);
    for (int i = 0; i < cfg->n_instances; ++i) {
        if (check_instance(ctx, inst[i], i) != MRFV_OK) return bail(MRFV_EINVAL);
        if (inst[i].eos != inst[0].eos) {
            ctx->err = "every instance of a context needs the same equation of state";
            return bail(MRFV_EINVAL);
        }
        ctx->inst.push_back(inst[i]);
    }
    if (inst[0].eos == MRFV_TAIT &&
        (cfg->scheme != MRFV_ROE_WENO5 || (cfg->batched && cfg->dtype == MRFV_F32))) {
        ctx->err = "Tait's equation runs on the plain kernels with the Roe-WENO5 flux";
        return bail(MRFV_EINVAL);
    }
    for (int i = 0; i < cfg->n_instances; ++i) ctx->viscous = ctx->viscous || inst[i].mu > 0.0;
    if (ctx->viscous && cfg->batched && cfg->dtype == MRFV_F32) {
        ctx->err = "the viscous terms run on the plain kernels, not on the fused FP32 path";
        return bail(MRFV_EINVAL);
    }
    ctx->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&ctx->device) != hipSuccess ||
        static_totals_scratch(ctx->device, &ctx->d_static_totals) != hipSuccess) {
        ctx->err = "cannot resolve the static totals scratch";
        return bail(MRFV_EHIP);
    }
    const size_t cap = cfg->slot_capacity, es = elem_size(ctx);
    ctx->lists_cap = 2 * cfg->n_instances + 10 * cfg->slot_capacity + 16;
    ctx->prim_batch = 128;
    ctx->lvl_bound.assign(MAX_LEVELS, 0);
    for (int i = 0; i < cfg->n_instances; ++i) {
        int64_t n = (int64_t)inst[i].n0[0] * inst[i].n0[1] * inst[i].n0[2];
        for (int l = 0; l <= inst[i].lmax && l < MAX_LEVELS; ++l, n *= 8) ctx->lvl_bound[l] += n;
    }
    if (cfg->batched < 0 || cfg->batched > 2) return bail(MRFV_EINVAL);
    std::vector<InstDev> id(cfg->n_instances);
    for (int i = 0; i < cfg->n_instances; ++i) {
        const mrfv_instance &p = inst[i];
        id[i] = InstDev{p.gamma, p.B, p.cfl, p.eps, p.scale_rho, p.scale_E, p.dx0, p.lmax,
                        {p.n0[0], p.n0[1], p.n0[2]}, {p.bc[0], p.bc[1], p.bc[2]}, p.adapt,
                        DETAIL_BAND_DEFAULT, {p.gravity[0], p.gravity[1], p.gravity[2]},
                        (p.gravity[0] != 0.0 || p.gravity[1] != 0.0 || p.gravity[2] != 0.0) ? 1 : 0,
                        p.eos, p.tait_A, p.tait_rho0, p.mu};
    }
#define ALLOC(ptr, bytes)                                                                  \
    if (hipMalloc((void **)&(ptr), (bytes)) != hipSuccess) {                                \
        ctx->err = "hipMalloc failed";                                                     \
        return bail(MRFV_ENOMEM);                                                          \
    }
    ALLOC(ctx->d_inst, sizeof(InstDev) * id.size());
    for (int i = 0; i < cfg->n_instances; ++i)
        for (int a = 0; a < 3; ++a) {
            if (inst[i].bc[a] != MRFV_BC_PERIODIC) ctx->bounded = true;
            if (inst[i].bc[a] == MRFV_BC_SYMMETRY || inst[i].bc[a] == MRFV_BC_FIXED)
                ctx->tb.ext_bc = ctx->tb2.ext_bc = true;
        }
    {
        // fixed-value halo states, conservative in the context dtype
        bool any = false;
        for (int i = 0; i < cfg->n_instances; ++i)
            for (int a = 0; a < 3; ++a) any = any || inst[i].bc[a] == MRFV_BC_FIXED;
        if (any) {
            const size_t per = (size_t)6 * MAX_LEVELS * 4 * 5;
            std::vector<double> h(per * cfg->n_instances, 0.0);
            for (int i = 0; i < cfg->n_instances; ++i) {
                const mrfv_instance &p = inst[i];
                for (int a = 0; a < 3; ++a) {
                    if (p.bc[a] != MRFV_BC_FIXED) continue;
                    for (int sd = 0; sd < 2; ++sd)
                        for (int l = 0; l <= p.lmax; ++l)
                            for (int ly = 0; ly < 4; ++ly) {
                                const double *w = p.bc_fixed + (((size_t)(2 * a + sd) * (p.lmax + 1) + l) * 4 + ly) * 5;
                                double *u = h.data() + per * i + (((size_t)(2 * a + sd) * MAX_LEVELS + l) * 4 + ly) * 5;
                                u[0] = w[0];
                                for (int c = 0; c < 3; ++c) u[1 + c] = w[0] * w[1 + c];
                                u[4] = p.eos == MRFV_TAIT ? 0.0
                                                          : (w[4] + p.gamma * p.B) / (p.gamma - 1.0) +
                                                                0.5 * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
                            }
                }
            }
            ALLOC(ctx->d_bcfix, h.size() * es);
            std::vector<float> f(h.begin(), h.end());
            const void *src = es == sizeof(double) ? (const void *)h.data() : (const void *)f.data();
            if (hipMemcpy(ctx->d_bcfix, src, h.size() * es, hipMemcpyHostToDevice) != hipSuccess) {
                ctx->err = "hipMemcpy of the fixed-value boundary states failed";
                return bail(MRFV_EHIP);
            }
            ctx->tb.bcfix = ctx->tb2.bcfix = ctx->d_bcfix;
        }
    }
    ALLOC(ctx->d_err, sizeof(int32_t));
    if (!(cfg->batched && cfg->dtype == MRFV_F32)) {
        ALLOC(ctx->d_D, cap * 3 * 5 * CELLS_I * es);
    } else {
        ALLOC(ctx->d_W, cap * 5 * CELLS_P * es);    // second and third state buffers of the
        ALLOC(ctx->d_W2, cap * 5 * CELLS_P * es);   // fused stages
    }
    ALLOC(ctx->d_desc, 2 * N_DESC * sizeof(int32_t));
    ALLOC(ctx->d_desc_g, 2 * N_DESC * sizeof(int32_t));
    ALLOC(ctx->d_gate, 2 * sizeof(int32_t));
    if (hipHostMalloc((void **)&ctx->h_flags, 2 * cap, 0) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_err, 2 * sizeof(int32_t), 0) != hipSuccess) {
        ctx->err = "hipHostMalloc failed";
        return bail(MRFV_ENOMEM);
    }
    std::fill(ctx->h_flags, ctx->h_flags + 2 * cap, (int8_t)0);
    ctx->h_err[0] = ctx->h_err[1] = 0;
    ALLOC(ctx->d_FF, cap * 6 * 5 * FACE * es);
    ALLOC(ctx->d_blockred, cap * std::max(5, 3 * cfl_slabs()) * sizeof(double));
    if (ctx->viscous) ALLOC(ctx->d_viscred, cap * sizeof(double));
    ALLOC(ctx->d_det, cap * sizeof(double));
    ALLOC(ctx->d_det4, cap * details_parts() * sizeof(double));
    ALLOC(ctx->d_recheck, (2 + cap * details_parts()) * sizeof(int32_t));
    ALLOC(ctx->d_flags, cap);
    ALLOC(ctx->d_slots, cap * sizeof(int32_t));
    ALLOC(ctx->d_slots2, cap * sizeof(int32_t));
    ALLOC(ctx->d_prim, (size_t)ctx->prim_batch * 5 * CELLS_I * sizeof(double));
    ALLOC(ctx->tb.meta, cap * sizeof(BlockMeta));
    ALLOC(ctx->tb.child, cap * 8 * sizeof(int32_t));
    ALLOC(ctx->tb.nbr, cap * 27 * sizeof(int32_t));
    ALLOC(ctx->tb.lists, (size_t)ctx->lists_cap * sizeof(int32_t));
#undef ALLOC
    if (hipMemcpy(ctx->d_inst, id.data(), sizeof(InstDev) * id.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemset(ctx->d_err, 0, sizeof(int32_t)) != hipSuccess ||
        hipMemset(ctx->d_det, 0, cap * sizeof(double)) != hipSuccess ||
        hipMemset(ctx->d_gate, 0, 2 * sizeof(int32_t)) != hipSuccess ||
        hipMemset(ctx->d_recheck, 0, 2 * sizeof(int32_t)) != hipSuccess)
        return bail(MRFV_EHIP);
    ctx->topo.reset(cfg->slot_capacity, ctx->inst);
    *out = ctx;
    return MRFV_OK;
}

int mrfv_destroy(mrfv_ctx *ctx) {
    if (!ctx) return MRFV_EINVAL;
    if (ctx->stream) hipStreamSynchronize(ctx->stream);
    else hipDeviceSynchronize();
    drop_graphs(ctx);
    if (ctx->gstream) hipStreamDestroy(ctx->gstream);
    if (ctx->side) {
        hipStreamSynchronize(ctx->side);
        hipStreamDestroy(ctx->side);
    }
    if (ctx->ev_prop) hipEventDestroy(ctx->ev_prop);
    if (ctx->h_flags) hipHostFree(ctx->h_flags);
    if (ctx->h_err) hipHostFree(ctx->h_err);
    if (ctx->h_logits) hipHostFree(ctx->h_logits);
    {
        void *pp[] = {ctx->d_X, ctx->d_logits, ctx->tb2.meta, ctx->tb2.child, ctx->tb2.nbr,
                      ctx->tb2.lists, ctx->d_desc2};
        for (void *p : pp)
            if (p) hipFree(p);
    }
    void *ptrs[] = {ctx->d_inst, ctx->d_err, ctx->d_D, ctx->d_W, ctx->d_W2, ctx->d_FF, ctx->d_Fp, ctx->d_H0, ctx->d_ACC,
                    ctx->d_blockred, ctx->d_viscred, ctx->d_bcfix, ctx->d_det, ctx->d_det4,
                    ctx->d_recheck, ctx->d_flags, ctx->d_slots, ctx->d_slots2, ctx->d_prim, ctx->tb.meta, ctx->tb.child,
                    ctx->tb.nbr, ctx->tb.lists, ctx->d_desc, ctx->d_desc_g, ctx->d_gate};
    for (void *p : ptrs)
        if (p) hipFree(p);
    for (hipEvent_t e : ctx->ev_free) hipEventDestroy(e);
    for (hipEvent_t e : ctx->ev_pairs) hipEventDestroy(e);
    delete ctx;
    return MRFV_OK;
}

const char *mrfv_last_error(const mrfv_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int64_t mrfv_state_bytes(const mrfv_ctx *ctx) {
    return ctx ? (int64_t)ctx->cfg.slot_capacity * 5 * CELLS_P * (int64_t)elem_size(ctx) : -1;
}

int64_t mrfv_interior_bytes(const mrfv_ctx *ctx) {
    return ctx ? (int64_t)ctx->cfg.slot_capacity * 5 * CELLS_I * (int64_t)elem_size(ctx) : -1;
}

int mrfv_init_blocks(mrfv_ctx *ctx, mrfv_ic_fn ic, void *user, void *U) {
    if (!ctx) return MRFV_EINVAL;
    if (!ic || !U) return fail(ctx, MRFV_EINVAL, "init_blocks: null callback or U");
    return ctx->cfg.dtype == MRFV_F64 ? do_init<double>(ctx, ic, user, (double *)U)
                                      : do_init<float>(ctx, ic, user, (float *)U);
}

int mrfv_fill_halos(mrfv_ctx *ctx, void *U) {
    CALL(need_init(ctx));
    if (!U) return fail(ctx, MRFV_EINVAL, "fill_halos: null U");
    return ctx->cfg.dtype == MRFV_F64 ? do_fill<double>(ctx, (double *)U, 1 << 20)
                                      : do_fill<float>(ctx, (float *)U, 1 << 20);
}

int mrfv_rhs_stage(mrfv_ctx *ctx, const void *U, void *L) {
    CALL(need_init(ctx));
    if (!U || !L) return fail(ctx, MRFV_EINVAL, "rhs_stage: null pointer");
    return ctx->cfg.dtype == MRFV_F64 ? do_rhs<double>(ctx, (const double *)U, (double *)L)
                                      : do_rhs<float>(ctx, (const float *)U, (float *)L);
}

int mrfv_rk_update(mrfv_ctx *ctx, int32_t stage, const double *dt_dev, void *U, void *U0,
                   const void *L) {
    CALL(need_init(ctx));
    if (stage < 0 || stage > 2) return fail(ctx, MRFV_EINVAL, "rk_update: stage must be 0..2");
    if (!dt_dev || !U || !U0 || !L) return fail(ctx, MRFV_EINVAL, "rk_update: null pointer");
    return ctx->cfg.dtype == MRFV_F64
               ? do_update<double>(ctx, stage, dt_dev, (double *)U, (double *)U0, (const double *)L)
               : do_update<float>(ctx, stage, dt_dev, (float *)U, (float *)U0, (const float *)L);
}

int mrfv_mr_project(mrfv_ctx *ctx, void *U) {
    CALL(need_init(ctx));
    if (!U) return fail(ctx, MRFV_EINVAL, "mr_project: null U");
    return ctx->cfg.dtype == MRFV_F64 ? do_project<double>(ctx, (double *)U)
                                      : do_project<float>(ctx, (float *)U);
}

int mrfv_mr_predict(mrfv_ctx *ctx, void *U, const int32_t *slots_host, int32_t n) {
    CALL(need_init(ctx));
    if (!U || (n > 0 && !slots_host)) return fail(ctx, MRFV_EINVAL, "mr_predict: null pointer");
    if (n < 0 || n > ctx->cfg.slot_capacity) return fail(ctx, MRFV_EINVAL, "mr_predict: bad count");
    for (int i = 0; i < n; ++i) {
        const int s = slots_host[i];
        if (s < 0 || s >= ctx->cfg.slot_capacity || !ctx->topo.block(s).alive ||
            ctx->topo.block(s).level == 0)
            return fail(ctx, MRFV_EINVAL, "mr_predict: slot is not a live block with a parent");
    }
    return ctx->cfg.dtype == MRFV_F64 ? do_predict<double>(ctx, (double *)U, slots_host, n)
                                      : do_predict<float>(ctx, (float *)U, slots_host, n);
}

int mrfv_mr_flag(mrfv_ctx *ctx, const void *U, int8_t *flags_dev, double *det_dev) {
    CALL(need_init(ctx));
    if (!U || !flags_dev || !det_dev) return fail(ctx, MRFV_EINVAL, "mr_flag: null pointer");
    return ctx->cfg.dtype == MRFV_F64
               ? do_details_flags<double>(ctx, (const double *)U, flags_dev, det_dev)
               : do_details_flags<float>(ctx, (const float *)U, flags_dev, det_dev);
}

int mrfv_set_detail_band(mrfv_ctx *ctx, double band) {
    if (!ctx) return MRFV_EINVAL;
    if (!(band >= 0.0)) return fail(ctx, MRFV_EINVAL, "set_detail_band: band must be >= 0");
    std::vector<InstDev> id(ctx->inst.size());
    HIP_OK(hipStreamSynchronize(ctx->stream));
    HIP_OK(hipMemcpy(id.data(), ctx->d_inst, sizeof(InstDev) * id.size(), hipMemcpyDeviceToHost));
    for (InstDev &d : id) d.detail_band = band;
    HIP_OK(hipMemcpy(ctx->d_inst, id.data(), sizeof(InstDev) * id.size(), hipMemcpyHostToDevice));
    return MRFV_OK;
}

int mrfv_cfl_dt(mrfv_ctx *ctx, const void *U, double *dt_dev) {
    CALL(need_init(ctx));
    if (!U || !dt_dev) return fail(ctx, MRFV_EINVAL, "cfl_dt: null pointer");
    if (ctx->cfg.dtype == MRFV_F64)
        return do_cfl<double>(ctx, (const double *)U, dt_dev);
    return do_cfl<float>(ctx, (const float *)U, dt_dev);
}

int mrfv_totals(mrfv_ctx *ctx, const void *U, double *tot_dev) {
    CALL(need_init(ctx));
    if (!U || !tot_dev) return fail(ctx, MRFV_EINVAL, "totals: null pointer");
    if (ctx->cfg.dtype == MRFV_F64)
        HIP_OK(launch_totals<double>((const double *)U, wlist(ctx, DESC_LEAVES), ctx->tb, ctx->d_inst,
                                     (int)ctx->inst.size(), ctx->d_blockred, tot_dev, ctx->stream));
    else
        HIP_OK(launch_totals<float>((const float *)U, wlist(ctx, DESC_LEAVES), ctx->tb, ctx->d_inst,
                                    (int)ctx->inst.size(), ctx->d_blockred, tot_dev, ctx->stream));
    return MRFV_OK;
}

int mrfv_totals_noalloc(mrfv_ctx *ctx, const void *U, double *tot_dev) {
    CALL(need_init(ctx));
    if (!U || !tot_dev) return fail(ctx, MRFV_EINVAL, "totals_noalloc: null pointer");
    if (ctx->cfg.slot_capacity > static_totals_slots())
        return fail(ctx, MRFV_EINVAL,
                    "totals_noalloc: slot capacity " + std::to_string(ctx->cfg.slot_capacity) +
                        " exceeds the static scratch (" + std::to_string(static_totals_slots()) +
                        " slots); use mrfv_totals");
    int cur = -1;
    HIP_OK(hipGetDevice(&cur));
    if (cur != ctx->device)
        return fail(ctx, MRFV_ESTATE, "totals_noalloc: the context's device is not current");
    // every listed slot's partials are written before they are read: nothing to clear
    if (ctx->cfg.dtype == MRFV_F64)
        HIP_OK(launch_totals<double>((const double *)U, wlist(ctx, DESC_LEAVES), ctx->tb, ctx->d_inst,
                                     (int)ctx->inst.size(), ctx->d_static_totals, tot_dev, ctx->stream));
    else
        HIP_OK(launch_totals<float>((const float *)U, wlist(ctx, DESC_LEAVES), ctx->tb, ctx->d_inst,
                                    (int)ctx->inst.size(), ctx->d_static_totals, tot_dev, ctx->stream));
    return MRFV_OK;
}

int mrfv_commit_flags(mrfv_ctx *ctx, const int8_t *flags_host, int32_t *new_slots_host,
                      int32_t *n_new) {
    CALL(need_init(ctx));
    if (!flags_host) return fail(ctx, MRFV_EINVAL, "commit_flags: null flags");
    std::vector<int32_t> fresh;
    CALL(commit(ctx, flags_host, fresh));
    if (new_slots_host) std::copy(fresh.begin(), fresh.end(), new_slots_host);
    if (n_new) *n_new = (int32_t)fresh.size();
    return MRFV_OK;
}

int mrfv_step(mrfv_ctx *ctx, void *U, void *U0, void *L, double *dt_dev) {
    CALL(need_init(ctx));
    if (!U || !U0 || !L || !dt_dev) return fail(ctx, MRFV_EINVAL, "step: null pointer");
    return ctx->cfg.dtype == MRFV_F64
               ? do_step<double>(ctx, (double *)U, (double *)U0, (double *)L, dt_dev)
               : do_step<float>(ctx, (float *)U, (float *)U0, (float *)L, dt_dev);
}

int mrfv_step_lts(mrfv_ctx *ctx, void *U, void *U0, void *L, double *dt_dev,
                  int64_t *cell_updates_host) {
    CALL(need_init(ctx));
    if (!U || !U0 || !dt_dev) return fail(ctx, MRFV_EINVAL, "step_lts: null pointer");
    if (ctx->viscous) return fail(ctx, MRFV_EINVAL, "step_lts: the viscous terms run with the global step only");
    for (const auto &p : ctx->inst)
        if (p.lmax != ctx->inst[0].lmax)
            return fail(ctx, MRFV_EINVAL, "step_lts: every instance needs the same lmax");
    return ctx->cfg.dtype == MRFV_F64
               ? do_step_lts<double>(ctx, (double *)U, (double *)U0, (double *)L, dt_dev, cell_updates_host)
               : do_step_lts<float>(ctx, (float *)U, (float *)U0, (float *)L, dt_dev, cell_updates_host);
}

int mrfv_run(mrfv_ctx *ctx, void *U, void *U0, void *L, double *dt_dev, int32_t n_steps,
             int64_t *leaf_cells_host) {
    CALL(need_init(ctx));
    if (!U || !U0 || !L || !dt_dev) return fail(ctx, MRFV_EINVAL, "run: null pointer");
    if (n_steps < 0) return fail(ctx, MRFV_EINVAL, "run: n_steps must be >= 0");
    int64_t cells = 0;
    const int rc = ctx->cfg.dtype == MRFV_F64
                       ? do_run<double>(ctx, (double *)U, (double *)U0, (double *)L, dt_dev, n_steps, &cells)
                       : do_run<float>(ctx, (float *)U, (float *)U0, (float *)L, dt_dev, n_steps, &cells);
    if (leaf_cells_host) *leaf_cells_host = cells;
    return rc;
}

int mrfv_check(mrfv_ctx *ctx) {
    if (!ctx) return MRFV_EINVAL;
    int32_t e = 0;
    HIP_OK(hipMemcpyAsync(&e, ctx->d_err, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    if (e) {
        HIP_OK(hipMemsetAsync(ctx->d_err, 0, sizeof(int32_t), ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
        return fail(ctx, MRFV_ENONPHYS, "non-physical state (rho<=0, p+B<=0 or NaN)");
    }
    return MRFV_OK;
}

int mrfv_stats(mrfv_ctx *ctx, int64_t *out) {
    if (!ctx || !out) return MRFV_EINVAL;
    out[0] = ctx->topo.count();
    out[1] = ctx->lists.all_leaves_cnt;
    out[2] = (int64_t)ctx->lists.all_leaves_cnt * CELLS_I;
    out[3] = ctx->lists.max_level;
    return MRFV_OK;
}

int mrfv_get_blocks(mrfv_ctx *ctx, int64_t *info, int32_t *n) {
    if (!ctx || !n) return MRFV_EINVAL;
    const std::vector<int> order = ctx->topo.alive_sorted();
    *n = (int32_t)order.size();
    if (info) {
        for (size_t k = 0; k < order.size(); ++k) {
            const HostBlock &b = ctx->topo.block(order[k]);
            int64_t *r = info + 8 * k;
            r[0] = order[k];
            r[1] = b.inst;
            r[2] = b.level;
            r[3] = b.bx;
            r[4] = b.by;
            r[5] = b.bz;
            r[6] = b.leaf ? 1 : 0;
            r[7] = (int64_t)b.morton;
        }
    }
    return MRFV_OK;
}

int mrfv_refine_block(mrfv_ctx *ctx, void *U, int32_t inst, int32_t level, int32_t bx,
                      int32_t by, int32_t bz) {
    CALL(need_init(ctx));
    if (!U || inst < 0 || inst >= (int)ctx->inst.size())
        return fail(ctx, MRFV_EINVAL, "refine_block: bad argument");
    const int s = ctx->topo.find(inst, level, bx, by, bz);
    if (s < 0 || !ctx->topo.block(s).leaf || level >= ctx->inst[inst].lmax)
        return fail(ctx, MRFV_EINVAL, "refine_block: not a refinable leaf");
    CALL(mrfv_fill_halos(ctx, U));
    std::vector<int> created;
    if (!ctx->topo.refine(s, &created)) return fail(ctx, MRFV_ENOMEM, "slot capacity exhausted");
    CALL(upload_tables(ctx));
    std::vector<int32_t> c32(created.begin(), created.end());
    return ctx->cfg.dtype == MRFV_F64 ? do_predict<double>(ctx, (double *)U, c32.data(), 8)
                                      : do_predict<float>(ctx, (float *)U, c32.data(), 8);
}

int mrfv_coarsen_block(mrfv_ctx *ctx, int32_t inst, int32_t level, int32_t bx, int32_t by,
                       int32_t bz) {
    CALL(need_init(ctx));
    if (inst < 0 || inst >= (int)ctx->inst.size())
        return fail(ctx, MRFV_EINVAL, "coarsen_block: bad instance");
    const int s = ctx->topo.find(inst, level, bx, by, bz);
    if (s < 0 || ctx->topo.block(s).leaf) return fail(ctx, MRFV_EINVAL, "coarsen_block: not a parent");
    for (int o = 0; o < 8; ++o)
        if (!ctx->topo.block(ctx->topo.block(s).child[o]).leaf)
            return fail(ctx, MRFV_EINVAL, "coarsen_block: children are not all leaves");
    ctx->topo.coarsen(s);
    return upload_tables(ctx);
}

int mrfv_features(mrfv_ctx *ctx, const void *U, float *X_dev, int32_t *slots_host, int32_t *n) {
    CALL(need_init(ctx));
    if (!U || !X_dev || !n) return fail(ctx, MRFV_EINVAL, "features: null pointer");
    const HostLists &L = ctx->lists;
    *n = L.all_leaves_cnt;
    if (slots_host)
        std::copy(L.data.begin() + L.all_leaves_off, L.data.begin() + L.all_leaves_off + L.all_leaves_cnt,
                  slots_host);
    if (ctx->cfg.dtype == MRFV_F64)
        HIP_OK(launch_features<double>((const double *)U, wlist(ctx, DESC_LEAVES), ctx->tb, ctx->d_inst,
                                       X_dev, ctx->stream));
    else
        HIP_OK(launch_features<float>((const float *)U, wlist(ctx, DESC_LEAVES), ctx->tb, ctx->d_inst,
                                      X_dev, ctx->stream));
    return MRFV_OK;
}

int mrfv_set_proposer(mrfv_ctx *ctx, mrfv_mlp *mlp, int32_t mode) {
    if (!ctx) return MRFV_EINVAL;
    if (mode < 0 || mode > 2 || (mode == 1 && !mlp))
        return fail(ctx, MRFV_EINVAL, "set_proposer: mode 0 (off), 1 (network) or 2 (persistence)");
    if (mode != 0 && ctx->inst[0].eos == MRFV_TAIT)
        return fail(ctx, MRFV_EINVAL, "set_proposer: the features assume the stiffened gas");
    const size_t cap = ctx->cfg.slot_capacity;
    if (mode != 0 && !ctx->tb2.meta) {
        auto al = [&](void **p, size_t bytes) { return hipMalloc(p, bytes) == hipSuccess; };
        if (!al((void **)&ctx->tb2.meta, cap * sizeof(BlockMeta)) ||
            !al((void **)&ctx->tb2.child, cap * 8 * sizeof(int32_t)) ||
            !al((void **)&ctx->tb2.nbr, cap * 27 * sizeof(int32_t)) ||
            !al((void **)&ctx->tb2.lists, (size_t)ctx->lists_cap * sizeof(int32_t)) ||
            !al((void **)&ctx->d_desc2, 2 * N_DESC * sizeof(int32_t)) ||
            !al((void **)&ctx->d_X, cap * 192 * sizeof(float)) ||
            !al((void **)&ctx->d_logits, cap * 3 * sizeof(float)))
            return fail(ctx, MRFV_ENOMEM, "set_proposer: device memory");
        if (hipHostMalloc((void **)&ctx->h_logits, cap * 3 * sizeof(float), 0) != hipSuccess)
            return fail(ctx, MRFV_ENOMEM, "set_proposer: pinned memory");
        HIP_OK(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
        HIP_OK(hipEventCreateWithFlags(&ctx->ev_prop, hipEventDisableTiming));
    }
    ctx->mlp = mlp;
    ctx->prop_mode = mode;
    ctx->p_net_due = true;
    return MRFV_OK;
}

int mrfv_fused_stage(mrfv_ctx *ctx, int32_t stage, const double *dt_dev, void *Uin, void *Uout,
                     void *U0, int32_t restrict_parents) {
    CALL(need_init(ctx));
    if (!(ctx->cfg.batched && ctx->cfg.dtype == MRFV_F32))
        return fail(ctx, MRFV_EINVAL, "fused_stage: batched FP32 contexts only");
    if (stage < 0 || stage > 2) return fail(ctx, MRFV_EINVAL, "fused_stage: stage must be 0..2");
    if (!dt_dev || !Uin || !Uout || !U0) return fail(ctx, MRFV_EINVAL, "fused_stage: null pointer");
    if (Uin == Uout) return fail(ctx, MRFV_EINVAL, "fused_stage: Uin and Uout must differ");
    const bool par = ctx->lists.parents_needed;
    if (par) CALL(do_project<float>(ctx, (float *)Uin, true));
    CALL(do_fill<float>(ctx, (float *)Uin, 1 << 20, FILL_MISSING_FACES, par));
    return do_stage_fused(ctx, stage, dt_dev, (const float *)Uin, (float *)Uout, (float *)U0,
                          restrict_parents != 0);
}

int mrfv_rhs_variant(mrfv_ctx *ctx, int32_t set, int32_t *n_variants, int32_t *shapes) {
    if (!ctx) return MRFV_EINVAL;
    const int n = rhs_variants(ctx->cfg.scheme);
    if (n_variants) *n_variants = n;
    if (shapes)
        for (int v = 0; v < n; ++v)
            rhs_variant_shape(ctx->cfg.scheme, v, shapes + 4 * v, shapes + 4 * v + 1, shapes + 4 * v + 2,
                              shapes + 4 * v + 3);
    if (set >= n) return fail(ctx, MRFV_EINVAL, "rhs_variant: index out of range");
    if (set >= 0 && set != ctx->rhs_variant) {
        ctx->rhs_variant = set;
        drop_graphs(ctx);   // captured graphs hold the old launch shape
    }
    return ctx->rhs_variant;
}

int mrfv_autotune(mrfv_ctx *ctx, void *U, void *U0, double *dt_dev, int32_t reps, float *ms_host,
                  int32_t *choice) {
    CALL(need_init(ctx));
    if (!U || !U0 || !dt_dev) return fail(ctx, MRFV_EINVAL, "autotune: null pointer");
    if (!(ctx->cfg.batched && ctx->cfg.dtype == MRFV_F32))
        return fail(ctx, MRFV_EINVAL, "autotune: only the batched FP32 path has launch variants");
    if (reps < 1 || reps > 1000) return fail(ctx, MRFV_EINVAL, "autotune: reps must be 1..1000");
    float *X = (float *)U, *W = (float *)ctx->d_W;
    hipStream_t st = ctx->stream;
    // a valid first stage: CFL step, restriction, fills; each variant then runs stage 0
    // from U into the second state buffer W (U, the state, is not written)
    HIP_OK(launch_cfl<float>(X, wlist(ctx, DESC_LEAVES), ctx->tb, ctx->d_inst, (int)ctx->inst.size(),
                             ctx->d_blockred, dt_dev, st));
    CALL(do_project<float>(ctx, X));
    CALL(do_fill<float>(ctx, X, 1 << 20, FILL_MISSING_FACES));
    const WorkList wl = wlist(ctx, DESC_LEAVES, 1 << 30);
    hipEvent_t a, b;
    HIP_OK(hipEventCreate(&a));
    HIP_OK(hipEventCreate(&b));
    int best = -1;
    float best_ms = 0.f;
    for (int v = 0; v < rhs_variants(ctx->cfg.scheme); ++v) {
        HIP_OK(launch_rhs_update_f32(ctx->cfg.scheme, v, 0, dt_dev, X, W, (float *)U0, wl, ctx->tb, ctx->d_inst,
                                     (float *)ctx->d_FF, ctx->d_err, 0, nullptr, st));
        HIP_OK(hipEventRecord(a, st));
        for (int r = 0; r < reps; ++r)
            HIP_OK(launch_rhs_update_f32(ctx->cfg.scheme, v, 0, dt_dev, X, W, (float *)U0, wl, ctx->tb, ctx->d_inst,
                                         (float *)ctx->d_FF, ctx->d_err, 0, nullptr, st));
        HIP_OK(hipEventRecord(b, st));
        HIP_OK(hipEventSynchronize(b));
        float ms = 0.f;
        HIP_OK(hipEventElapsedTime(&ms, a, b));
        ms /= reps;
        if (ms_host) ms_host[v] = ms;
        if (best < 0 || ms < best_ms) {
            best = v;
            best_ms = ms;
        }
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (best != ctx->rhs_variant) {
        ctx->rhs_variant = best;
        drop_graphs(ctx);
    }
    if (choice) *choice = best;
    return MRFV_OK;
}

int mrfv_step_timing(mrfv_ctx *ctx, double *out) {
    if (!ctx || !out) return MRFV_EINVAL;
    out[0] = (double)ctx->h_steps;
    out[1] = ctx->h_wait_ms;
    out[2] = ctx->h_commit_ms;
    out[3] = ctx->h_predict_ms;
    return MRFV_OK;
}

int mrfv_last_flags(mrfv_ctx *ctx, int8_t *flags_host) {
    if (!ctx || !flags_host) return MRFV_EINVAL;
    HIP_OK(hipStreamSynchronize(ctx->stream));
    const int8_t *hf = ctx->h_flags + (size_t)ctx->last_half * ctx->cfg.slot_capacity;
    std::copy(hf, hf + ctx->cfg.slot_capacity, flags_host);
    return MRFV_OK;
}

int mrfv_proposer_stats(mrfv_ctx *ctx, int64_t *out, double *build_ms) {
    if (!ctx || !out) return MRFV_EINVAL;
    out[0] = ctx->p_steps;
    out[1] = ctx->p_hits;
    for (int c = 0; c < 3; ++c) {
        out[2 + 3 * c] = ctx->p_tp[c];
        out[3 + 3 * c] = ctx->p_fp[c];
        out[4 + 3 * c] = ctx->p_fn[c];
    }
    out[11] = ctx->p_staged;
    out[12] = ctx->p_adopted;
    out[13] = ctx->p_net_runs;
    if (build_ms) *build_ms = ctx->p_build_ms;
    return MRFV_OK;
}

int mrfv_enable_kernel_timing(mrfv_ctx *ctx, int32_t on) {
    if (!ctx) return MRFV_EINVAL;
    ctx->timing = on != 0;
    return MRFV_OK;
}

int mrfv_kernel_time(mrfv_ctx *ctx, int64_t *launches, double *total_ms, int64_t *cells) {
    if (!ctx) return MRFV_EINVAL;
    HIP_OK(hipStreamSynchronize(ctx->stream));
    for (size_t i = 0; i + 1 < ctx->ev_pairs.size(); i += 2) {
        float ms = 0.f;
        HIP_OK(hipEventElapsedTime(&ms, ctx->ev_pairs[i], ctx->ev_pairs[i + 1]));
        ctx->t_ms += ms;
        ctx->t_launches += 1;
        ctx->t_cells += ctx->ev_cells[i / 2];
        ctx->ev_free.push_back(ctx->ev_pairs[i]);
        ctx->ev_free.push_back(ctx->ev_pairs[i + 1]);
    }
    ctx->ev_pairs.clear();
    ctx->ev_cells.clear();
    if (launches) *launches = ctx->t_launches;
    if (total_ms) *total_ms = ctx->t_ms;
    if (cells) *cells = ctx->t_cells;
    return MRFV_OK;
}

}  // extern "C"
