// mrfv_internal.h -- declarations shared by the library's host code and its HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mrfv.h"

namespace mrfv {

constexpr int NI = 16;               // interior cells per block edge
constexpr int HW = 4;                // halo layers per side
constexpr int NP = NI + 2 * HW;      // padded edge (24)
constexpr int CELLS_P = NP * NP * NP;    // 13824
constexpr int CELLS_I = NI * NI * NI;    // 4096
constexpr int FACE = NI * NI;            // 256

// Per-slot block description on the device (32 bytes).
struct BlockMeta {
    int32_t inst, level, bx, by, bz;
    int32_t parent;   // parent slot, -1 on level 0
    int32_t leaf;     // 1 = leaf
    int32_t zg;       // bit (2*axis + side): block touches a zero-gradient boundary there
};

// Per-instance parameters on the device.
struct InstDev {
    double gamma, B, cfl, eps, scale_rho, scale_E, dx0;
    int32_t lmax, n0[3], bc[3], adapt;
};

// Device-resident topology tables, rebuilt after every change of the tree.
struct DevTables {
    BlockMeta *meta = nullptr;   // [cap]
    int32_t *child = nullptr;    // [cap][8], -1 when absent
    int32_t *nbr = nullptr;      // [cap][27] same-level neighbour slot; -1 absent, -2 outside
    int32_t *lists = nullptr;    // concatenated work lists (see HostLists)
};

// Work lists, concatenated in DevTables::lists (host copy).  The array starts with the
// per-instance leaf ranges: data[i] = offset (into data) of instance i's leaves,
// data[n_inst + i] = their count; the instance ranges are contiguous parts of the
// all-leaves list, which is sorted by (instance, level, Morton id).
struct HostLists {
    std::vector<int32_t> data;
    int max_level = 0;
    // per level: all blocks, non-leaf blocks, leaves
    std::vector<int32_t> lvl_off, lvl_cnt, par_off, par_cnt, leaf_off, leaf_cnt;
    int32_t all_leaves_off = 0, all_leaves_cnt = 0;      // leaves of every level
    int32_t all_blocks_off = 0, all_blocks_cnt = 0;      // every block
    int32_t fine_off = 0, fine_cnt = 0;                  // every block with level >= 1
};

// ---------------------------------------------------------------- host topology ------
struct HostBlock {
    int32_t inst = 0, level = 0, bx = 0, by = 0, bz = 0;
    int32_t parent = -1;
    int32_t child[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
    bool leaf = true, alive = false;
    uint64_t morton = 0;
};

class Topology {
  public:
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

// --------------------------------------------------------------- kernel launchers ----
// All launchers enqueue on `st` and return hipGetLastError().
template <typename T>
hipError_t launch_prim2cons(const double *prim, const int32_t *slots, int n, T *U,
                            const BlockMeta *meta, const InstDev *inst, hipStream_t st);
template <typename T>
hipError_t launch_fill_halos(T *U, const int32_t *list, int n, const DevTables &tb,
                             int leaf_faces, hipStream_t st);
template <typename T>
hipError_t launch_project(T *U, const int32_t *list, int n, const DevTables &tb,
                          hipStream_t st);
template <typename T>
hipError_t launch_predict(T *U, const int32_t *list, int n, const DevTables &tb,
                          hipStream_t st);
template <typename T>
hipError_t launch_details(const T *U, const int32_t *list, int n, const DevTables &tb,
                          const InstDev *inst, double *det, hipStream_t st);
hipError_t launch_flags(const int32_t *list, int n, const DevTables &tb, const InstDev *inst,
                        const double *det, int8_t *flags, hipStream_t st);
template <typename T>
hipError_t launch_cfl(const T *U, const int32_t *leaves, int n, const DevTables &tb,
                      const InstDev *inst, int n_inst, double *blockmax, double *dt,
                      hipStream_t st);
template <typename T>
hipError_t launch_totals(const T *U, const int32_t *leaves, int n, const DevTables &tb,
                         const InstDev *inst, int n_inst, double *blocksum, double *tot,
                         hipStream_t st);
template <typename T>
hipError_t launch_flux(const T *U, const int32_t *leaves, int n, const DevTables &tb,
                       const InstDev *inst, T *D, T *FF, hipStream_t st);
template <typename T>
hipError_t launch_ff_restrict(T *FF, const int32_t *parents, int n, const DevTables &tb,
                              hipStream_t st);
template <typename T>
hipError_t launch_reflux(T *D, const T *FF, const int32_t *leaves, int n,
                         const DevTables &tb, hipStream_t st);
template <typename T>
hipError_t launch_combine(const T *D, T *L, const int32_t *leaves, int n,
                          const DevTables &tb, const InstDev *inst, hipStream_t st);
template <typename T>
hipError_t launch_update(int stage, const double *dt, T *U, T *U0, const T *L,
                         const int32_t *leaves, int n, const DevTables &tb,
                         const InstDev *inst, int32_t *err, hipStream_t st);
hipError_t launch_rhs_update_f32(int stage, const double *dt, float *U, float *U0,
                                 const int32_t *leaves, int n, const DevTables &tb,
                                 const InstDev *inst, float *FF, int32_t *err, hipStream_t st);
template <typename T>
hipError_t launch_reflux_update(int stage, const double *dt, T *U, const T *FF,
                                const int32_t *leaves, int n, const DevTables &tb,
                                const InstDev *inst, hipStream_t st);

}  // namespace mrfv

// ---------------------------------------------------------------- context -------------
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
    int32_t *d_err = nullptr;          // device error word
    void *d_D = nullptr;               // flux differences [cap][3][5][16^3]
    void *d_FF = nullptr;              // boundary face fluxes [cap][6][5][16][16]
    double *d_blockred = nullptr;      // [cap][5] per-block partial reductions
    double *d_det = nullptr;           // [cap]
    int8_t *d_flags = nullptr;         // [cap]
    int32_t *d_slots = nullptr;        // [cap] scratch slot list
    double *d_prim = nullptr;          // IC staging [batch][5][16^3]
    int prim_batch = 0;
    int lists_cap = 0;
    // kernel timing
    bool has_jumps = false;            // some leaf has a non-leaf same-level face neighbour
    bool timing = false;
    std::vector<hipEvent_t> ev_free;   // event pool
    std::vector<hipEvent_t> ev_pairs;  // recorded (start, stop) pairs not yet read
    std::vector<int64_t> ev_cells;
    int64_t t_launches = 0, t_cells = 0;
    double t_ms = 0.0;
};
