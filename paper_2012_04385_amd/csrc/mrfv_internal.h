// mrfv_internal.h -- declarations shared by the library's host code and its HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <unordered_map>
#include <map>
#include <vector>

#include "../../include/mrfv.h"

namespace mrfv {

constexpr int NI = 16;               // interior cells per block edge
constexpr int HW = 4;                // halo layers per side
constexpr int NP = NI + 2 * HW;      // padded edge (24)
constexpr int CELLS_P = NP * NP * NP;    // 13824
constexpr int CELLS_I = NI * NI * NI;    // 4096
constexpr int FACE = NI * NI;            // 256

// Per-slot block description on the device (40 bytes).
struct BlockMeta {
    int32_t inst, level, bx, by, bz;
    int32_t parent;   // parent slot, -1 on level 0
    int32_t leaf;     // 1 = leaf
    int32_t zg;       // bit (2*axis + side): block touches a non-periodic boundary there;
                      // bit (6 + 2*axis + side): that boundary is a symmetry plane;
                      // bit (12 + 2*axis + side): it has fixed values
    int32_t srestr;   // 1: leaf on level >= 1 without a non-leaf same-level face neighbour
                      // (no jump correction): the fused stage writes its restriction into
                      // the parent's octant
    int32_t lpos;     // position in the all-leaves list (-1: not a leaf)
    int32_t pmask;    // non-leaf blocks: bit i set when a stage's prediction of a finer halo
                      // reads halo region i of this block (make_region's index of the 26)
};

// Per-instance parameters on the device.
struct InstDev {
    double gamma, B, cfl, eps, scale_rho, scale_E, dx0;
    int32_t lmax, n0[3], bc[3], adapt;
    double detail_band;   // slabs with |detail - eps_l| <= band are evaluated again exactly
    double gravity[3];    // source term S(U) = (0, rho g, rho v . g)
    int32_t has_source;   // gravity is not the zero vector
    int32_t eos;          // 0 stiffened gas, 1 Tait (p = B ((rho/rho0)^gamma - 1) + A)
    double tait_A, tait_rho0;
    double mu;            // dynamic viscosity (0: no viscous terms)
};
constexpr double DETAIL_BAND_DEFAULT = 1e-9;

// Device-resident topology tables, rebuilt after every change of the tree.
struct DevTables {
    BlockMeta *meta = nullptr;   // [cap]
    int32_t *child = nullptr;    // [cap][8], -1 when absent
    int32_t *nbr = nullptr;      // [cap][27] same-level neighbour slot; -1 absent, -2 outside
    int32_t *lists = nullptr;    // concatenated work lists (see HostLists)
    const void *bcfix = nullptr; // fixed-value halo states (context dtype, conservative):
                                 // [inst][6 sides][MAX_LEVELS][4 layers][5]; null if none
    bool ext_bc = false;         // some instance has a symmetry or fixed-value side
};

// A work list of block slots.  Eager launches pass the offset and count from the host;
// graph-captured launches pass a device descriptor {offset, count} that the host rewrites
// whenever the tree changes, so a captured graph stays valid.  Kernels loop over the list
// with a grid stride, so any grid size is correct.
struct WorkList {
    const int32_t *base = nullptr;   // device list array
    const int32_t *desc = nullptr;   // device {offset, count}, or null
    int32_t off = 0, n = 0;          // host offset and count when desc is null
    int grid = 0;                    // workgroups to launch (0: skip the launch)
    __device__ __forceinline__ int count() const { return desc ? desc[1] : n; }
    __device__ __forceinline__ int32_t at(int i) const { return base[(desc ? desc[0] : off) + i]; }
};

// XCD-aware item order for a one-dimensional grid of `total` workgroups handling `m` <= total
// items: the chip hands workgroup w to XCD w mod 8, so item order x * ceil(m / 8) + w / 8 gives
// each XCD one contiguous range of the list (Morton-ordered blocks: spatial neighbours and
// siblings share an L2).  Returns m for workgroups without an item.  A total that is not a
// multiple of 8 keeps the identity order (the covering argument needs total >= 8 ceil(m / 8)).
constexpr int N_XCD = 8;
__device__ __forceinline__ int xcd_item(int w, int total, int m) {
    if (total % N_XCD) return w < m ? w : m;
    const int per = (m + N_XCD - 1) / N_XCD, l = w / N_XCD;
    const int i = (w % N_XCD) * per + l;
    return l < per && i < m ? i : m;
}
inline int round_xcd(int grid) { return (grid + N_XCD - 1) / N_XCD * N_XCD; }

// Signal speeds |v_d| + c, d = 0, 1, 2, of one cell for the CFL condition, FP64 with explicit
// fused multiply-adds, so that every kernel evaluating it (the CFL pass, the last stage of
// a step) rounds alike and their block maxima agree bitwise.
__device__ __forceinline__ void cfl_speeds(double r, double m0, double m1, double m2, double E,
                                           double gamma, double B, double s[3]) {
    const double ir = 1.0 / r;
    const double k2 = fma(m2, m2, fma(m1, m1, m0 * m0));
    const double p = fma(gamma - 1.0, fma(-0.5 * k2, ir, E), -gamma * B);
    const double cs = sqrt(gamma * (p + B) * ir);
    s[0] = fma(fabs(m0), ir, cs);
    s[1] = fma(fabs(m1), ir, cs);
    s[2] = fma(fabs(m2), ir, cs);
}
// The same for Tait's equation, c^2 = gamma B / rho0 (rho / rho0)^(gamma - 1).
__device__ __forceinline__ void cfl_speeds_tait(double r, double m0, double m1, double m2,
                                                double gamma, double B, double rho0, double s[3]) {
    const double ir = 1.0 / r;
    const double cs = sqrt(gamma * B / rho0 * pow(r / rho0, gamma - 1.0));
    s[0] = fma(fabs(m0), ir, cs);
    s[1] = fma(fabs(m1), ir, cs);
    s[2] = fma(fabs(m2), ir, cs);
}
constexpr int CFL_SLABS = 4;   // per-block CFL maxima: [slot][CFL_SLABS][3]

// Work lists, concatenated in DevTables::lists (host copy).  The array starts with the
// per-instance leaf ranges: data[i] = offset (into data) of instance i's leaves,
// data[n_inst + i] = their count; the instance ranges are contiguous parts of the
// all-leaves list, which is sorted by (instance, level, Morton id).
struct HostLists {
    std::vector<int32_t> data;
    int max_level = 0;
    // per level: all blocks, non-leaf blocks, leaves
    std::vector<int32_t> lvl_off, lvl_cnt, par_off, par_cnt, leaf_off, leaf_cnt, jleaf_off, jleaf_cnt,
        j26_off, j26_cnt, pfill_off, pfill_cnt, pproj_off, pproj_cnt;
    int32_t all_leaves_off = 0, all_leaves_cnt = 0;      // leaves of every level
    // descriptor table {offset, count} per list, mirrored on the device (graph launches)
    std::vector<int32_t> desc;
    int32_t all_blocks_off = 0, all_blocks_cnt = 0;      // every block
    int32_t fine_off = 0, fine_cnt = 0;                  // every block with level >= 1
    int32_t jcorr_off = 0, jcorr_cnt = 0;                // leaves the jump correction changes
    int32_t pars_off = 0, pars_cnt = 0;                  // every non-leaf block
    // no non-leaf block on level >= 1 has a halo region without a same-level neighbour or
    // on a zero-gradient side: filling the parents' halos is copies only, in any order
    bool pars_copy_only = false;
    // some leaf face reads a parent-derived value inside a stage: no same-level neighbour
    // (predicted halo) or a non-leaf same-level neighbour (restricted interior)
    bool parents_needed = false;
    // per level: every child of every block in the par / pproj list has meta.srestr (a
    // restriction pass that skips those octants has nothing to do)
    std::vector<uint8_t> par_srestr, pproj_srestr;
};

// ---------------------------------------------------------------- host topology ------
struct HostBlock {
    int32_t inst = 0, level = 0, bx = 0, by = 0, bz = 0;
    int32_t parent = -1;
    int32_t child[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
    bool leaf = true, alive = false;
    uint64_t morton = 0;
};

// One recorded tree edit (for undoing a speculative commit).
struct TreeOp {
    int kind;        // 1 refine, -1 coarsen
    int slot;        // refined leaf / coarsened parent
    int child[8];    // slots of the created / removed children
};

class Topology {
  public:
    // Apply flags (per slot: 1 refine, -1 coarsen) to the leaves; records the edits.
    bool commit(const int8_t *flags, std::vector<TreeOp> *ops, std::vector<int> *fresh);
    // Undo recorded edits (reverse order); restores slots and the free list exactly.
    void undo(const std::vector<TreeOp> &ops);
    void reset(int capacity, const std::vector<mrfv_instance> &inst);
    int add_block(int inst, int level, int bx, int by, int bz);   // -1 when full
    int find(int inst, int level, int bx, int by, int bz) const;
    bool refine(int slot, std::vector<int> *created);              // false when full
    void coarsen(int parent_slot);
    void remove_block(int slot);
    // Builds host copies of the device tables and work lists.
    void build(std::vector<BlockMeta> &meta, std::vector<int32_t> &child,
               std::vector<int32_t> &nbr, HostLists &lists) const;
    int capacity() const { return (int)blocks_.size(); }
    int count() const { return n_alive_; }
    const HostBlock &block(int s) const { return blocks_[s]; }
    int shadow(int inst) const { return shadow_[inst]; }
    std::vector<int> alive_sorted() const;   // by (inst, level, morton)

  private:
    static uint64_t key(int inst, int level, int bx, int by, int bz);
    std::vector<HostBlock> blocks_;
    std::vector<int> free_;
    std::unordered_map<uint64_t, int> map_;
    std::vector<mrfv_instance> inst_;
    std::vector<int> shadow_;
    int n_alive_ = 0;
};

uint64_t morton_encode(int shadow, int level, int bx, int by, int bz);

// Descriptor indices of the work lists (DevTables lists + the device descriptor table).
constexpr int MAX_LEVELS = 13;
// DESC_JCORR: leaves with a non-leaf same-level face neighbour (the jump correction
// changes their boundary cells after the fused stage)
// DESC_PARS: every non-leaf block, all levels
constexpr int DESC_LEAVES = 0, DESC_ALL = 1, DESC_FINE = 2, DESC_JCORR = 3, DESC_PARS = 4;
constexpr int DESC_PER_LEVEL = 7;
constexpr int desc_lvl(int l) { return 5 + DESC_PER_LEVEL * l; }
constexpr int desc_par(int l) { return 6 + DESC_PER_LEVEL * l; }
constexpr int desc_leaf(int l) { return 7 + DESC_PER_LEVEL * l; }
// leaves of level l with at least one face that has no same-level neighbour or lies on a
// zero-gradient boundary: the only leaves whose halos a fused stage must fill
constexpr int desc_jleaf(int l) { return 8 + DESC_PER_LEVEL * l; }
// leaves of level l with at least one of the 26 halo regions lacking a same-level
// neighbour or on a zero-gradient boundary (filled before the details)
constexpr int desc_jleaf26(int l) { return 9 + DESC_PER_LEVEL * l; }
// non-leaf blocks of level l whose halo a stage's predictions read: parents of leaves
// with a face lacking a same-level neighbour, and parents of such blocks that lack a
// same-level neighbour in some region themselves
constexpr int desc_pfill(int l) { return 10 + DESC_PER_LEVEL * l; }
// non-leaf blocks of level l whose interior a stage reads: the stage's prediction
// sources, their non-leaf same-level neighbours (copied into their halos), non-leaf
// same-level face neighbours of leaves, and the non-leaf descendants of all of these
constexpr int desc_pproj(int l) { return 11 + DESC_PER_LEVEL * l; }
constexpr int N_DESC = 5 + DESC_PER_LEVEL * MAX_LEVELS;

// Halo fill modes, two flags: FACES restricts the fill to the 6 face regions, 3 layers
// deep (all the flux stencils read); MISSING to the regions without a same-level
// neighbour or on a zero-gradient boundary (the other regions are read in place from
// the neighbour's interior by the fused stage and the details).
// FILL_RHO_E limits any mode to the density and energy components (the details read
// nothing else).  FILL_PRESENT (with FILL_FACES) copies only: faces without a same-level
// neighbour keep their values (the integrated jump halos of local time stepping).
// FILL_MASKED (with FILL_ALL, for the prediction sources of a stage) fills only the
// regions in the block's pmask.
enum FillMode { FILL_ALL = 0, FILL_FACES = 1, FILL_MISSING = 2, FILL_MISSING_FACES = 3, FILL_RHO_E = 4,
                FILL_PRESENT = 8, FILL_MASKED = 16 };

// --------------------------------------------------------------- kernel launchers ----
// All launchers enqueue on `st` and return hipGetLastError().
template <typename T>
hipError_t launch_prim2cons(const double *prim, const int32_t *slots, int n, T *U,
                            const BlockMeta *meta, const InstDev *inst, hipStream_t st);
template <typename T>
hipError_t launch_fill_halos(T *U, const WorkList &wl, const DevTables &tb, FillMode mode,
                             hipStream_t st);
template <typename T>
hipError_t launch_project(T *U, const WorkList &wl, const DevTables &tb, hipStream_t st,
                          int qmask = 31,          // bit q: restrict component q
                          bool skip_srestr = false);   // leave octants of srestr children
template <typename T>
hipError_t launch_predict(T *U, const int32_t *list, int n, const DevTables &tb,
                          hipStream_t st);
template <typename T>
hipError_t launch_details(const T *U, const WorkList &wl, const DevTables &tb,
                          const InstDev *inst, double *det4, int32_t *recheck, hipStream_t st);
int details_parts();   // detail maxima per block in det4 (one per slab)
// flags (and det of blocks on level >= 1) from the slab maxima; flags_host / err_host
// (may be null): host-memory copies of the flags and of the error word err; gate (may be
// null; graph launches): {tree changed, launch parity}: the host copies go to the half
// given by the parity ([2][cap] flags, [2] error words) and a refine or coarsen sets gate[0]
hipError_t launch_flags(const WorkList &wl, const DevTables &tb, const InstDev *inst,
                        const double *det4, double *det, int8_t *flags, int8_t *flags_host,
                        const int32_t *err, int32_t *err_host, int32_t *gate, int cap,
                        hipStream_t st);
// per-block maxima, then dt per instance; with gate words (step graphs) the second launch
// also writes desc_g = desc, counts zeroed when gate[0] is set
template <typename T>
hipError_t launch_cfl(const T *U, const WorkList &leaves, const DevTables &tb,
                      const InstDev *inst, int n_inst, double *blockmax, double *dt,
                      hipStream_t st, int32_t *gate = nullptr, const int32_t *desc = nullptr,
                      int32_t *desc_g = nullptr, int n_desc = 0);
int cfl_slabs();      // z-slab maxima per block in the CFL reduction
// Static device scratch of the allocation-free totals: its capacity in slots, and its
// device address on `device` (looked up once, with that device current).
int static_totals_slots();
hipError_t static_totals_scratch(int device, double **ptr);
// the per-block pass of the CFL step alone, over any list of leaves
template <typename T>
hipError_t launch_cfl_blocks(const T *U, const WorkList &wl, const DevTables &tb,
                             const InstDev *inst, double *blockmax, hipStream_t st);
// Viscous terms (kernels_visc.hip): the viscous flux subtracted from the plain flux
// kernel's differences D and face planes FF of the listed leaves, and the viscous bound on
// the time step (dt[inst] = min(dt[inst], cfl 3/16 dx_lmax^2 / (mu max 1/rho))) for the
// instances with mu > 0; blockmax: one double per leaf.
template <typename T>
hipError_t launch_visc(const T *U, const WorkList &wl, const DevTables &tb, const InstDev *inst,
                       T *D, T *FF, hipStream_t st);
template <typename T>
hipError_t launch_visc_dt(const T *U, const WorkList &leaves, const DevTables &tb,
                          const InstDev *inst, int n_inst, double *blockmax, double *dt,
                          hipStream_t st);
template <typename T>
hipError_t launch_totals(const T *U, const WorkList &leaves, const DevTables &tb,
                         const InstDev *inst, int n_inst, double *blocksum, double *tot,
                         hipStream_t st);
template <typename T>
hipError_t launch_flux(int scheme, const T *U, const WorkList &leaves, const DevTables &tb,
                       const InstDev *inst, T *D, T *FF, hipStream_t st);
template <typename T>
hipError_t launch_ff_restrict(T *FF, const WorkList &parents, const DevTables &tb,
                              hipStream_t st);
template <typename T>
hipError_t launch_reflux(T *D, const T *FF, const WorkList &leaves, const DevTables &tb,
                         hipStream_t st);
template <typename T>
hipError_t launch_combine(const T *D, T *L, const WorkList &leaves, const DevTables &tb,
                          const InstDev *inst, const T *U, hipStream_t st);
template <typename T>
hipError_t launch_update(int stage, const double *dt, T *U, T *U0, const T *L,
                         const WorkList &leaves, const DevTables &tb, const InstDev *inst,
                         int32_t *err, hipStream_t st);
// Fused stage: reads the state from Uin (same-level neighbours' interiors directly, the
// own halo elsewhere) and writes the new interior state to Uout != Uin.
// scheme: flux kernel (mrfv_scheme); variant: launch shape index in [0, rhs_variants(scheme))
// (all give the same result).
// restrict_parents: leaves with meta.srestr also write the restriction of their new state
// (all components) into their parent's octant of Uout.
// stage < 0: no update; Uout (a padded field) receives the interior flux divergence
// L = -sum_d dF_d / dx + S (local time stepping), and with restrict_parents its
// restriction into the parents' octants of Uout; U0 is not touched, cflmax must be null.
hipError_t launch_rhs_update_f32(int scheme, int variant, int stage, const double *dt, const float *Uin,
                                 float *Uout, float *U0, const WorkList &leaves, const DevTables &tb,
                                 const InstDev *inst, float *FF, int32_t *err, int restrict_parents,
                                 double *cflmax, hipStream_t st);   // cflmax: null, or CFL block maxima out
int rhs_variants(int scheme);
int rhs_default_variant(int scheme);   // the shape fastest on the measured trees
void rhs_variant_shape(int scheme, int v, int *gp, int *tpb, int *wpe, int *ptr);
template <typename T>
hipError_t launch_reflux_update(int stage, const double *dt, T *U, const T *FF,
                                const WorkList &leaves, const DevTables &tb,
                                const InstDev *inst, hipStream_t st);
// Local time stepping (kernels_lts.hip).  F: padded flux divergence [cap][5][24^3];
// H0: stage-start state of the halo cells of jump faces [cap][6][5][lts_halo_slab()];
// ACC: time-integrated boundary face fluxes [cap][6][5][16][16] (the layout of FF).
template <typename T>
hipError_t launch_lts_combine(const T *D, T *F, const WorkList &leaves, const DevTables &tb,
                              const InstDev *inst, const T *U, hipStream_t st);
template <typename T>
hipError_t launch_lts_update(int stage, const double *dt, T *U, T *U0, T *H0, const T *F,
                             const T *FF, T *ACC, const WorkList &leaves, const DevTables &tb,
                             const InstDev *inst, int32_t *err, hipStream_t st);
template <typename T>
hipError_t launch_lts_adjust(T *U, const T *ACC, const WorkList &leaves, const DevTables &tb,
                             const InstDev *inst, hipStream_t st);
template <typename T>
hipError_t launch_lts_zero(T *ACC, const WorkList &leaves, const DevTables &tb, int lo_end,
                           hipStream_t st);
int lts_halo_slab();
template <typename T>
hipError_t launch_features(const T *U, const WorkList &wl, const DevTables &tb, const InstDev *inst,
                           float *X, hipStream_t st);

}  // namespace mrfv

// ---------------------------------------------------------------- context -------------
struct mrfv_mlp;
namespace mrfv {
// The proposer network's forward pass queued on a given stream; logits [N][3] FP32.
int mlp_forward_on(mrfv_mlp *mm, hipStream_t st, const float *X, int N, float *logits);
}  // namespace mrfv
// Which launches a captured step graph holds: two words of per-level list emptiness.
using GraphKey = std::pair<uint64_t, uint64_t>;

struct mrfv_ctx {
    mrfv_config cfg{};
    std::vector<mrfv_instance> inst;
    hipStream_t stream = nullptr;
    std::string err;
    bool initialised = false;
    mrfv::Topology topo;
    mrfv::HostLists lists;
    mrfv::DevTables tb;
    mrfv::InstDev *d_inst = nullptr;
    int device = -1;                   // the HIP device current at mrfv_create
    double *d_static_totals = nullptr; // that device's static totals scratch (not owned)
    int32_t *d_err = nullptr;          // device error word
    void *d_W = nullptr, *d_W2 = nullptr;   // second and third padded state buffers
                                            // (fused FP32 stages: U -> W -> W2 -> U)
    void *d_D = nullptr;               // flux differences [cap][3][5][16^3]
    void *d_FF = nullptr;              // boundary face fluxes [cap][6][5][16][16]
    void *d_Fp = nullptr, *d_H0 = nullptr, *d_ACC = nullptr;   // local time stepping, on first use
    double *d_blockred = nullptr;      // [cap][5] per-block partial reductions
    double *d_viscred = nullptr;       // [cap] per-leaf max 1/rho (viscous contexts)
    void *d_bcfix = nullptr;           // fixed-value halo states (see DevTables::bcfix)
    double *d_det = nullptr;           // [cap]
    double *d_det4 = nullptr;          // [cap][details_parts()] slab maxima of the details
    int32_t *d_recheck = nullptr;      // [2 + cap * details_parts()]: count, done count, list of
                                       // slabs whose detail lies near the threshold (zero between launches)
    int8_t *d_flags = nullptr;         // [cap]
    int32_t *d_desc = nullptr;         // [N_DESC][2] list descriptors (graph launches)
    hipStream_t gstream = nullptr;     // capture stream of the step graphs
    hipGraphExec_t graph = nullptr;    // graph being instantiated
    std::map<GraphKey, hipGraphExec_t> graphs;   // step graphs (gate, CFL, three RK stages,
                                                 // adaptation up to the flags) by graph key,
                                                 // valid for (gU, gU0, gdt)
    void *gU = nullptr, *gU0 = nullptr;
    const double *gdt = nullptr;
    std::vector<int64_t> lvl_bound;    // most blocks any level can hold
    // learned refinement proposer
    mrfv_mlp *mlp = nullptr;
    int prop_mode = 0;                 // 0 off, 1 network, 2 persistence (no change)
    float *d_X = nullptr, *d_logits = nullptr;
    float *h_logits = nullptr;         // pinned
    int8_t *h_flags = nullptr;         // pinned [2][cap], judge flags (halves: launch parity)
    int32_t *h_err = nullptr;          // pinned [2]
    int32_t *d_gate = nullptr;         // {tree changed by the last flags, launch parity}
    int32_t *d_desc_g = nullptr;       // descriptors as gated for the current step graph
    int64_t graph_launches = 0;        // step graphs launched (parity of the next: +1)
    int last_half = 0;                 // half of h_flags / h_err the last step wrote
    std::vector<int8_t> proposal;      // per slot
    mrfv::DevTables tb2;               // staging tables built from the proposal
    int32_t *d_desc2 = nullptr;
    mrfv::HostLists lists2;
    std::vector<mrfv::BlockMeta> s_meta;
    std::vector<int32_t> s_child, s_nbr;
    bool staged = false, staged_jumps = false;
    hipStream_t side = nullptr;        // staging uploads
    hipEvent_t ev_prop = nullptr;      // proposal copied to the host
    int64_t p_steps = 0, p_hits = 0, p_tp[3] = {0, 0, 0}, p_fp[3] = {0, 0, 0}, p_fn[3] = {0, 0, 0};
    int64_t p_staged = 0, p_adopted = 0;
    bool p_net_due = true;             // the network runs on the next step (the last one changed the tree)
    int64_t p_net_runs = 0;            // steps on which the network ran
    double p_build_ms = 0.0;
    // host time of the adaptation phase of mrfv_step: waiting for the judged flags, tree
    // commit + table build + upload (or adoption of staged tables), prediction; steps
    double h_wait_ms = 0.0, h_commit_ms = 0.0, h_predict_ms = 0.0;
    int64_t h_steps = 0;
    int32_t *d_slots = nullptr;        // [cap] scratch slot list
    int32_t *d_slots2 = nullptr;       // [cap] second scratch slot list
    int rhs_variant = 0;               // launch shape of the fused kernel (default or autotuned)
    double *d_prim = nullptr;          // IC staging [batch][5][16^3]
    int prim_batch = 0;
    int lists_cap = 0;
    // kernel timing
    bool has_jumps = false;            // some leaf has a non-leaf same-level face neighbour
    bool viscous = false;              // some instance has mu > 0 (plain path only)
    bool bounded = false;              // some instance has a non-periodic axis
    bool capturing = false;            // recording a step graph
    // step graphs: the CFL pass takes the block maxima the previous step wrote after its
    // last stage (set by mrfv_run for a step that follows a step on the same tree)
    bool cfl_from_stage = false;
    // step graphs: the first stage's restriction skips the octants the previous step's last
    // stage restricted (set by mrfv_run for a step that follows a step on the same tree)
    bool restrict_from_stage = false;
    bool timing = false;
    std::vector<hipEvent_t> ev_free;   // event pool
    std::vector<hipEvent_t> ev_pairs;  // recorded (start, stop) pairs not yet read
    std::vector<int64_t> ev_cells;
    int64_t t_launches = 0, t_cells = 0;
    double t_ms = 0.0;
};
