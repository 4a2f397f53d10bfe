// abi.cpp -- C ABI of the library: context, tree bookkeeping and the order of kernel
// launches for initialisation (algo:Init) and the global time step (algo:ComputeLoop).
#include <hip/hip_runtime.h>

#include <algorithm>
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
    if (p.lmax < 0 || p.lmax > 12) return fail(ctx, MRFV_EINVAL, w + "lmax must be in [0,12]");
    for (int a = 0; a < 3; ++a) {
        if (p.n0[a] < 1 || ((int64_t)p.n0[a] << p.lmax) > 65535)
            return fail(ctx, MRFV_EINVAL, w + "n0 out of range");
        if (p.bc[a] != MRFV_BC_PERIODIC && p.bc[a] != MRFV_BC_ZEROGRAD)
            return fail(ctx, MRFV_EINVAL, w + "bc must be 0 or 1");
    }
    return MRFV_OK;
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
    HIP_OK(hipStreamSynchronize(st));   // host vectors die at return
    // jump faces exist when some leaf has a non-leaf same-level face neighbour
    ctx->has_jumps = false;
    const HostLists &L = ctx->lists;
    for (int t = 0; t < L.all_leaves_cnt && !ctx->has_jumps; ++t) {
        const int s = L.data[L.all_leaves_off + t];
        const int faces[6] = {12, 14, 10, 16, 4, 22};
        for (int f = 0; f < 6; ++f) {
            const int nb = nbr[(size_t)s * 27 + faces[f]];
            if (nb >= 0 && !ctx->topo.block(nb).leaf) { ctx->has_jumps = true; break; }
        }
    }
    return MRFV_OK;
}

const int32_t *dlist(const mrfv_ctx *ctx, int32_t off) { return ctx->tb.lists + off; }

template <typename T>
int do_project(mrfv_ctx *ctx, T *U) {
    const HostLists &L = ctx->lists;
    for (int l = L.max_level - 1; l >= 0; --l)
        HIP_OK(launch_project<T>(U, dlist(ctx, L.par_off[l]), L.par_cnt[l], ctx->tb, ctx->stream));
    return MRFV_OK;
}

// leaf_faces = 1 inside a stage: leaves get only the face layers the flux reads.
template <typename T>
int do_fill(mrfv_ctx *ctx, T *U, int max_level, int leaf_faces = 0) {
    const HostLists &L = ctx->lists;
    for (int l = 0; l <= std::min(max_level, L.max_level); ++l)
        HIP_OK(launch_fill_halos<T>(U, dlist(ctx, L.lvl_off[l]), L.lvl_cnt[l], ctx->tb, leaf_faces,
                                    ctx->stream));
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
    T *D = (T *)ctx->d_D, *FF = (T *)ctx->d_FF;
    hipEvent_t ev{};
    timing_begin(ctx, &ev);
    if (ctx->cfg.batched) {
        HIP_OK(launch_flux<T>(U, dlist(ctx, L.all_leaves_off), L.all_leaves_cnt, ctx->tb,
                              ctx->d_inst, D, FF, ctx->stream));
    } else {
        for (int l = 0; l <= L.max_level; ++l)
            HIP_OK(launch_flux<T>(U, dlist(ctx, L.leaf_off[l]), L.leaf_cnt[l], ctx->tb, ctx->d_inst,
                                  D, FF, ctx->stream));
    }
    timing_end(ctx, ev, (int64_t)L.all_leaves_cnt * CELLS_I);
    if (ctx->has_jumps) {
        for (int l = L.max_level - 1; l >= 0; --l)
            HIP_OK(launch_ff_restrict<T>(FF, dlist(ctx, L.par_off[l]), L.par_cnt[l], ctx->tb,
                                         ctx->stream));
        HIP_OK(launch_reflux<T>(D, FF, dlist(ctx, L.all_leaves_off), L.all_leaves_cnt, ctx->tb,
                                ctx->stream));
    }
    return MRFV_OK;
}

template <typename T>
int do_rhs(mrfv_ctx *ctx, const T *U, T *Lout) {
    CALL(do_flux<T>(ctx, U));
    const HostLists &L = ctx->lists;
    HIP_OK(launch_combine<T>((const T *)ctx->d_D, Lout, dlist(ctx, L.all_leaves_off),
                             L.all_leaves_cnt, ctx->tb, ctx->d_inst, ctx->stream));
    return MRFV_OK;
}

template <typename T>
int do_update(mrfv_ctx *ctx, int stage, const double *dt, T *U, T *U0, const T *Lb) {
    const HostLists &L = ctx->lists;
    HIP_OK(launch_update<T>(stage, dt, U, U0, Lb, dlist(ctx, L.all_leaves_off), L.all_leaves_cnt,
                            ctx->tb, ctx->d_inst, ctx->d_err, ctx->stream));
    return MRFV_OK;
}

// One stage of the batched path: fused rhs + update over all leaves, then the jump
// correction on the updated state.
int do_stage_fused(mrfv_ctx *ctx, int stage, const double *dt, float *U, float *U0) {
    const HostLists &L = ctx->lists;
    float *FF = (float *)ctx->d_FF;
    hipEvent_t ev{};
    timing_begin(ctx, &ev);
    HIP_OK(launch_rhs_update_f32(stage, dt, U, U0, dlist(ctx, L.all_leaves_off), L.all_leaves_cnt,
                                 ctx->tb, ctx->d_inst, FF, ctx->d_err, ctx->stream));
    timing_end(ctx, ev, (int64_t)L.all_leaves_cnt * CELLS_I);
    if (ctx->has_jumps) {
        for (int l = L.max_level - 1; l >= 0; --l)
            HIP_OK(launch_ff_restrict<float>(FF, dlist(ctx, L.par_off[l]), L.par_cnt[l], ctx->tb,
                                             ctx->stream));
        HIP_OK(launch_reflux_update<float>(stage, dt, U, FF, dlist(ctx, L.all_leaves_off),
                                           L.all_leaves_cnt, ctx->tb, ctx->d_inst, ctx->stream));
    }
    return MRFV_OK;
}

template <typename T>
int do_details_flags(mrfv_ctx *ctx, const T *U, int8_t *flags, double *det) {
    const HostLists &L = ctx->lists;
    HIP_OK(launch_details<T>(U, dlist(ctx, L.fine_off), L.fine_cnt, ctx->tb, ctx->d_inst, det,
                             ctx->stream));
    HIP_OK(launch_flags(dlist(ctx, L.all_blocks_off), L.all_blocks_cnt, ctx->tb, ctx->d_inst, det,
                        flags, ctx->stream));
    return MRFV_OK;
}

template <typename T>
int do_predict(mrfv_ctx *ctx, T *U, const int32_t *slots_host, int n) {
    if (n <= 0) return MRFV_OK;
    HIP_OK(hipMemcpyAsync(ctx->d_slots, slots_host, sizeof(int32_t) * n, hipMemcpyHostToDevice,
                          ctx->stream));
    HIP_OK(launch_predict<T>(U, ctx->d_slots, n, ctx->tb, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));   // slots_host may be a temporary
    return MRFV_OK;
}

int commit(mrfv_ctx *ctx, const int8_t *flags, std::vector<int32_t> &fresh) {
    std::vector<int> order = ctx->topo.alive_sorted();
    std::vector<int> coarsen, refine;
    for (int s : order) {
        const HostBlock &b = ctx->topo.block(s);
        if (!b.leaf) continue;
        if (flags[s] == 1) refine.push_back(s);
        if (flags[s] == -1 && (b.bx & 1) == 0 && (b.by & 1) == 0 && (b.bz & 1) == 0)
            coarsen.push_back(b.parent);
    }
    for (int p : coarsen) ctx->topo.coarsen(p);
    std::vector<int> created;
    for (int s : refine) {
        created.clear();
        if (!ctx->topo.refine(s, &created)) return fail(ctx, MRFV_ENOMEM, "slot capacity exhausted");
        fresh.insert(fresh.end(), created.begin(), created.end());
    }
    return upload_tables(ctx);
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
    std::vector<double> det(ctx->cfg.slot_capacity);
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
            HIP_OK(launch_details<T>(U, ctx->d_slots, (int)fresh.size(), ctx->tb, ctx->d_inst,
                                     ctx->d_det, ctx->stream));
            HIP_OK(hipMemcpyAsync(det.data(), ctx->d_det, sizeof(double) * det.size(),
                                  hipMemcpyDeviceToHost, ctx->stream));
            HIP_OK(hipStreamSynchronize(ctx->stream));
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

template <typename T>
int do_step(mrfv_ctx *ctx, T *U, T *U0, T *Lb, double *dt) {
    const HostLists &L0 = ctx->lists;
    HIP_OK(launch_cfl<T>(U, dlist(ctx, L0.all_leaves_off), L0.all_leaves_cnt, ctx->tb, ctx->d_inst,
                         (int)ctx->inst.size(), ctx->d_blockred, dt, ctx->stream));
    for (int s = 0; s < 3; ++s) {
        CALL(do_project<T>(ctx, U));
        CALL(do_fill<T>(ctx, U, 1 << 20, 1));
        if (ctx->cfg.batched && sizeof(T) == 4) {
            CALL(do_stage_fused(ctx, s, dt, (float *)U, (float *)U0));
        } else {
            CALL(do_rhs<T>(ctx, U, Lb));
            CALL(do_update<T>(ctx, s, dt, U, U0, Lb));
        }
    }
    bool adapt = false;
    for (const auto &p : ctx->inst) adapt = adapt || (p.adapt && p.lmax > 0);
    if (!adapt) return MRFV_OK;
    CALL(do_project<T>(ctx, U));
    CALL(do_fill<T>(ctx, U, 1 << 20));
    CALL(do_details_flags<T>(ctx, U, ctx->d_flags, ctx->d_det));
    std::vector<int8_t> flags(ctx->cfg.slot_capacity);
    int32_t errw = 0;
    HIP_OK(hipMemcpyAsync(flags.data(), ctx->d_flags, flags.size(), hipMemcpyDeviceToHost,
                          ctx->stream));
    HIP_OK(hipMemcpyAsync(&errw, ctx->d_err, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    if (errw) return fail(ctx, MRFV_ENONPHYS, "non-physical state (rho<=0, p+B<=0 or NaN)");
    std::vector<int32_t> fresh;
    CALL(commit(ctx, flags.data(), fresh));
    CALL(do_predict<T>(ctx, U, fresh.data(), (int)fresh.size()));
    return MRFV_OK;
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
    if (cfg->dtype != MRFV_F32 && cfg->dtype != MRFV_F64) return bail(MRFV_EINVAL);
    if (cfg->n_instances < 1 || cfg->n_instances > 4095) return bail(MRFV_EINVAL);
    if (cfg->slot_capacity < 1 || cfg->slot_capacity > (1 << 22)) return bail(MRFV_EINVAL);
    for (int i = 0; i < cfg->n_instances; ++i) {
        if (check_instance(ctx, inst[i], i) != MRFV_OK) return bail(MRFV_EINVAL);
        ctx->inst.push_back(inst[i]);
    }
    ctx->stream = (hipStream_t)hip_stream;
    const size_t cap = cfg->slot_capacity, es = elem_size(ctx);
    ctx->lists_cap = 2 * cfg->n_instances + 6 * cfg->slot_capacity + 16;
    ctx->prim_batch = 128;
    std::vector<InstDev> id(cfg->n_instances);
    for (int i = 0; i < cfg->n_instances; ++i) {
        const mrfv_instance &p = inst[i];
        id[i] = InstDev{p.gamma, p.B, p.cfl, p.eps, p.scale_rho, p.scale_E, p.dx0, p.lmax,
                        {p.n0[0], p.n0[1], p.n0[2]}, {p.bc[0], p.bc[1], p.bc[2]}, p.adapt};
    }
#define ALLOC(ptr, bytes)                                                                  \
    if (hipMalloc((void **)&(ptr), (bytes)) != hipSuccess) {                                \
        ctx->err = "hipMalloc failed";                                                     \
        return bail(MRFV_ENOMEM);                                                          \
    }
    ALLOC(ctx->d_inst, sizeof(InstDev) * id.size());
    ALLOC(ctx->d_err, sizeof(int32_t));
    ALLOC(ctx->d_D, cap * 3 * 5 * CELLS_I * es);
    ALLOC(ctx->d_FF, cap * 6 * 5 * FACE * es);
    ALLOC(ctx->d_blockred, cap * 5 * sizeof(double));
    ALLOC(ctx->d_det, cap * sizeof(double));
    ALLOC(ctx->d_flags, cap);
    ALLOC(ctx->d_slots, cap * sizeof(int32_t));
    ALLOC(ctx->d_prim, (size_t)ctx->prim_batch * 5 * CELLS_I * sizeof(double));
    ALLOC(ctx->tb.meta, cap * sizeof(BlockMeta));
    ALLOC(ctx->tb.child, cap * 8 * sizeof(int32_t));
    ALLOC(ctx->tb.nbr, cap * 27 * sizeof(int32_t));
    ALLOC(ctx->tb.lists, (size_t)ctx->lists_cap * sizeof(int32_t));
#undef ALLOC
    if (hipMemcpy(ctx->d_inst, id.data(), sizeof(InstDev) * id.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemset(ctx->d_err, 0, sizeof(int32_t)) != hipSuccess ||
        hipMemset(ctx->d_det, 0, cap * sizeof(double)) != hipSuccess)
        return bail(MRFV_EHIP);
    ctx->topo.reset(cfg->slot_capacity, ctx->inst);
    *out = ctx;
    return MRFV_OK;
}

int mrfv_destroy(mrfv_ctx *ctx) {
    if (!ctx) return MRFV_EINVAL;
    if (ctx->stream) hipStreamSynchronize(ctx->stream);
    else hipDeviceSynchronize();
    void *ptrs[] = {ctx->d_inst, ctx->d_err, ctx->d_D, ctx->d_FF, ctx->d_blockred, ctx->d_det,
                    ctx->d_flags, ctx->d_slots, ctx->d_prim, ctx->tb.meta, ctx->tb.child,
                    ctx->tb.nbr, ctx->tb.lists};
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

int mrfv_cfl_dt(mrfv_ctx *ctx, const void *U, double *dt_dev) {
    CALL(need_init(ctx));
    if (!U || !dt_dev) return fail(ctx, MRFV_EINVAL, "cfl_dt: null pointer");
    const HostLists &L = ctx->lists;
    if (ctx->cfg.dtype == MRFV_F64)
        HIP_OK(launch_cfl<double>((const double *)U, dlist(ctx, L.all_leaves_off), L.all_leaves_cnt,
                                  ctx->tb, ctx->d_inst, (int)ctx->inst.size(), ctx->d_blockred,
                                  dt_dev, ctx->stream));
    else
        HIP_OK(launch_cfl<float>((const float *)U, dlist(ctx, L.all_leaves_off), L.all_leaves_cnt,
                                 ctx->tb, ctx->d_inst, (int)ctx->inst.size(), ctx->d_blockred,
                                 dt_dev, ctx->stream));
    return MRFV_OK;
}

int mrfv_totals(mrfv_ctx *ctx, const void *U, double *tot_dev) {
    CALL(need_init(ctx));
    if (!U || !tot_dev) return fail(ctx, MRFV_EINVAL, "totals: null pointer");
    const HostLists &L = ctx->lists;
    if (ctx->cfg.dtype == MRFV_F64)
        HIP_OK(launch_totals<double>((const double *)U, dlist(ctx, L.all_leaves_off),
                                     L.all_leaves_cnt, ctx->tb, ctx->d_inst, (int)ctx->inst.size(),
                                     ctx->d_blockred, tot_dev, ctx->stream));
    else
        HIP_OK(launch_totals<float>((const float *)U, dlist(ctx, L.all_leaves_off),
                                    L.all_leaves_cnt, ctx->tb, ctx->d_inst, (int)ctx->inst.size(),
                                    ctx->d_blockred, tot_dev, ctx->stream));
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
