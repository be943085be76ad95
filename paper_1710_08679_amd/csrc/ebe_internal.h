// Internal declarations of the EBE library: the mesh handle, device buffers,
// error reporting and the kernel launchers shared between translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "ebe.h"

namespace ebe {

// Connectivity words carry the node id in the low 28 bits and the node's
// Dirichlet flags (x, y, z) in bits 28..30, so that a kernel that gathers a
// node also knows which of its DOFs are fixed without a second load.
constexpr int32_t kIdxBits = 28;
constexpr int32_t kIdxMask = (1 << kIdxBits) - 1;

void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

// Kernels move node rows of vectors in 16-byte pieces.
inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

#define EBE_TRY_HIP(call)                                                        \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      ::ebe::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),    \
                       __FILE__, __LINE__);                                      \
      return EBE_ERR_HIP;                                                        \
    }                                                                            \
  } while (0)

// Owned device allocation.
class DBuf {
 public:
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  ebe_status alloc(size_t bytes);        // no-op when already at least this large
  void release();
  template <class T> T* as() const { return static_cast<T*>(p_); }
  size_t bytes() const { return n_; }
 private:
  void* p_ = nullptr;
  size_t n_ = 0;
};

// An operator assembled into 3x3 blocks, in slices of kSliceRows rows: slice
// s has soff[s+1] - soff[s] slots (its longest row), slot j of row r is entry
// j * kSliceRows + r; short rows are padded with zero blocks whose column is
// the row itself.  Values value-major within a slot, so the rows of a
// wavefront read each value from one contiguous run.
struct AsmOp {
  DBuf soff;    // int32 [nslices+1]
  DBuf col;     // int32 [slots][kSliceRows] column id | fix bits
  DBuf val[2];  // [slots][9][kSliceRows] block values (row-major 3x3), per dtype (F64, F32)
  int64_t rows = 0, slots = 0;
  bool ready[2] = {false, false};
  // FP16 copy of the values divided by half_scale (the largest magnitude
  // over 2^14), for the coarse levels of a mixed solve with coarse_half set
  DBuf val16;
  double half_scale = 1.0;
  bool ready16 = false;
};

// Solver workspace; grown to the largest nrhs seen.
struct Workspace {
  int nrhs_cap = 0;
  // FP64 outer vectors [N][3][nrhs]
  DBuf r, p, q;
  // preconditioner vectors (FP32 or FP64) on levels 0, 1 and 2
  DBuf rb, ub, e0, p0, q0;
  DBuf r1, u1, e1, p1, q1;
  DBuf r2, u2, e2, p2, q2;
  // per-column scalars and reduction partials
  DBuf scal;      // double scalars (see solver.cpp for the slots)
  DBuf partials;  // block partial sums
  DBuf flags;     // int32 device flags
  DBuf counter;   // int32/uint32 arrival counters for last-block reductions
  int* host_flags = nullptr;  // pinned host mirror
  // Instantiated graphs of fixed runs of solver steps, keyed by everything
  // baked into their kernel arguments (buffer addresses, nrhs, step count).
  struct Graph {
    std::vector<uintptr_t> key;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<Graph> graphs;
  int64_t captures = 0;  // graphs captured so far (ebe_pcg_stats reports the count per solve)
};

// Element patches (patches.cpp): consecutive element ranges whose node sums
// fit in LDS.  Quadratic level: at most kPatchElems elements touching at most
// kPatchNodes nodes; 48 elements and 128 nodes fit a block of 2x2x2
// hexahedra of 6 tetrahedra (5^3 = 125 nodes) exactly, so on meshes in
// Morton order patches are compact blocks and fewer of their nodes are shared
// than with 64-element ranges that cut hexahedra apart.  Linear level: at most
// kLinPatchElems elements touching at most kLinPatchCorners corners (a linear
// element carries far less work, so its patches are larger).
#ifndef EBE_PATCH_ELEMS
#define EBE_PATCH_ELEMS 48
#endif
#ifndef EBE_PATCH_NODES
#define EBE_PATCH_NODES 128
#endif
#ifndef EBE_LIN_PATCH_ELEMS
#define EBE_LIN_PATCH_ELEMS 256
#endif
#ifndef EBE_LIN_PATCH_CORNERS
#define EBE_LIN_PATCH_CORNERS 128
#endif
#ifndef EBE_PATCH_THREADS
#define EBE_PATCH_THREADS 512
#endif
#ifndef EBE_PATCH_THREADS_F64
#define EBE_PATCH_THREADS_F64 256
#endif
constexpr int kSliceRows = 64;  // rows per slice of an assembled operator (AsmOp)
constexpr int kA2MaxRow = 800;  // longest level-2 row (blocks) whose sums fit 64 KB of LDS
constexpr int kPatchElems = EBE_PATCH_ELEMS;
constexpr int kPatchNodes = EBE_PATCH_NODES;
constexpr int kLinPatchElems = EBE_LIN_PATCH_ELEMS;
constexpr int kLinPatchCorners = EBE_LIN_PATCH_CORNERS;  // local ids are bytes: at most 256
constexpr int kPatchThreads = EBE_PATCH_THREADS;  // workgroup size cap of the patch kernels
// FP64 quadratic patches: smaller workgroups, so two fit per CU within the
// registers the FP64 element operator needs (two wavefronts per SIMD)
constexpr int kPatchThreadsF64 = EBE_PATCH_THREADS_F64;
static_assert(kPatchNodes <= 256 && kLinPatchCorners <= 256, "patch-local node ids are bytes");
// (x, K x) sums of the patch kernels: workgroup w adds its per-case sums to
// slot w % kGammaSlots (one 128-byte line each), and the last workgroup to
// finish folds the slots into the caller's result.
constexpr int kGammaSlots = 64;
constexpr size_t kGammaBytes = size_t(kGammaSlots) * EBE_MAX_RHS * sizeof(double) + 64;  // slots + counter

// Patch tables of one level (0: all nodes of the quadratic mesh, 1: corners).
struct PatchLevel {
  DBuf pelem;   // int32 [npatch+1] element offsets (patches are element ranges)
  int64_t npatch = 0;
  DBuf poff;    // int32 [npatch+1] entry offsets
  DBuf pnode;   // int32 [entries] node id | fix bits << 28 | shared << 31
  DBuf pslot;   // int32 [entries] staging slot of a shared entry, -1 otherwise
  DBuf snode;   // int32 [nshared] shared node id | fix bits << 28, increasing id
  DBuf soff;    // int32 [nshared+1] first staging slot of each shared node (its slots are consecutive)
  DBuf stage;   // staging buffer [nslots][3][nrhs] of the product's dtype
  int64_t nslots = 0, nshared = 0, entries = 0;
  int max_nodes = 0;
  // element node words [E][10] (quadratic) or [E][4] (linear): node id |
  // patch-local id << kPtabLocalShift; empty on meshes of 2^25 nodes or more
  DBuf ptab;
  // colouring of the patches (quadratic level): no two patches of a colour
  // share a node; cperm lists the patches colour by colour (increasing id
  // within a colour), colour c is cperm[coff[c] .. coff[c+1]); cword is
  // pnode with bit 31 meaning "an earlier colour wrote this node"
  DBuf cperm;
  DBuf cword;
  std::vector<int64_t> coff;
  // node-centric incidence lists of the quadratic patches (deterministic
  // form): pinc [E][10] element slots (element - patch's first) * 10 + a,
  // grouped by patch entry in element order; pistart [entries] the start of
  // an entry's list relative to its patch's first slot
  DBuf pinc;
  DBuf pistart;
};
// element node words: 25 bits of node id, 7 bits of patch-local id
constexpr int kPtabLocalShift = 25;
constexpr uint32_t kPtabIdMask = (1u << kPtabLocalShift) - 1;
static_assert(kPatchNodes <= 128 && kLinPatchCorners <= 128, "patch-local ids must fit 7 bits");

}  // namespace ebe

struct ebe_mesh {
  int64_t n_nodes = 0, n_vertices = 0, n_elem = 0;
  bool has_bc = false;
  // isoparametric (curved) quadratic elements: the quadratic level uses the
  // curved element kernel (gather form), xv holds every node
  bool curved = false;
  int device = 0;
  ebe::DBuf conn;       // int32 [E][10], packed (see kIdxBits)
  ebe::DBuf xv;         // double4 [Nv] corner coordinates (curved: [N], corners first; w unused)
  ebe::DBuf lame64;     // double2 [E] (lambda, mu)
  ebe::DBuf lame32;     // float2  [E]
  ebe::DBuf young;      // double [E]
  ebe::DBuf poisson;    // double [E]
  ebe::DBuf fix;        // uint8  [N] bit c = DOF c fixed
  ebe::DBuf edge_ends;  // int32 [N-Nv][2]
  ebe::DBuf v2e_off;    // int32 [Nv+1] corner -> incident edge nodes (CSR)
  ebe::DBuf v2e_idx;    // int32 [2 (N-Nv)]
  ebe::DBuf v2el_off;   // int32 [Nv+1] corner -> incident elements (CSR)
  ebe::DBuf v2el;       // int32 [4E] element * 4 + the corner's local index, by element
  // element patches of the two levels
  ebe::DBuf lconn;      // uint8 [E][16] quadratic-patch-local ids of the 10 nodes (padded to 16 bytes)
  ebe::DBuf lconn1;     // uint8 [E][4]  linear-patch-local ids of the 4 corners
  ebe::PatchLevel pl[2];
  ebe::DBuf gacc;       // kGammaBytes: (x, K x) slots, then the arrival counter; zero between products
  // EBE product form per [level][dtype F64, F32][nrhs]: one of the forms, or
  // EBE_FORM_AUTO (untuned: a fixed default)
  int8_t form[2][2][EBE_MAX_RHS + 1];
  // variant of the pipelined / coloured kernels per [level][dtype][nrhs]
  // (0: element geometry kept in LDS, 1: read per work-item), set by the tuner
  int8_t fvar[2][2][EBE_MAX_RHS + 1];
  ebe_mesh() {
    std::memset(form, EBE_FORM_AUTO, sizeof(form));
    std::memset(fvar, 0, sizeof(fvar));
  }
  // 3x3 block Jacobi: inverted symmetric blocks (xx yy zz yz zx xy), per level
  // (levels 0 and 1 with the material; level 2 with its operator)
  ebe::DBuf minv64[3], minv32[3];
  bool minv_ready = false;
  // geometry cache [E][16] per dtype (F64, F32): G, V, lambda, mu; filled on
  // first use by an entry point, dropped when the material changes
  ebe::DBuf geo[2];
  bool geo_ready[2] = {false, false};
  // assembled linear-level operator K1 over the corner graph (its edges are
  // the quadratic mesh's edge nodes); structure at creation, values on demand
  ebe::AsmOp k1;
  // level 2 (smoothed aggregation of the corner graph): aggregate of each
  // corner, coarse fix bits (a component is fixed when it is fixed at every
  // member), the smoothed prolongator P2 by fine rows (p2_width slots: the
  // aggregates of the corner and its neighbours, increasing, -1 padding; 3x3
  // blocks per slot, values with A2), its transpose as lists of P2 entries
  // per aggregate, and A2 = P2^T K1p P2 with its rows' lengths
  int64_t n_agg = 0;
  int32_t p2_width = 0;
  int32_t a2_maxlen = 0;  // longest row of A2 (blocks)
  ebe::DBuf agg;        // int32 [Nv]
  ebe::DBuf cfix;       // uint8 [Na]
  ebe::DBuf p2_col;     // int32 [Nv][p2_width]
  ebe::DBuf p2_val[2];  // [Nv][p2_width][9] per dtype (F64, F32)
  ebe::DBuf p2t_off;    // int32 [Na+1]
  ebe::DBuf p2t_idx;    // int32 [entries]: v * p2_width + slot
  ebe::DBuf a2_len;     // int32 [Na]
  ebe::AsmOp a2;
  ebe::Workspace ws;
};

namespace ebe {

// rows (nodes) of level 0 (quadratic mesh), 1 (corners) or 2 (aggregates)
inline int64_t level_rows(const ebe_mesh* m, int level) {
  return level == 0 ? m->n_nodes : (level == 1 ? m->n_vertices : m->n_agg);
}

// ---- kernel launchers (ebe_kernels.hip) -----------------------------------
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_ebe_p2(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y,
                         bool bc, hipStream_t s);
hipError_t launch_ebe_p1(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y,
                         bool bc, hipStream_t s);
// general form: order 2 (quadratic) or 1 (linear); mask_in: zero x's fixed
// DOFs while gathering; bc: zero y's fixed DOFs; add: y += K x instead of
// y = K x; the kernels do nothing when gate is non-null and *gate == 0 on the
// device.  gamma (optional, device [nrhs] FP64): gamma[r] += (x_r, K x_r)
// formed element by element.  The staging buffers must have been sized by
// ensure_stage.
// y = A2 x at level 2 (its values must be prepared: ensure_level2)
hipError_t launch_level2(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, bool mask_in, bool bc,
                         bool add, const int* gate, hipStream_t s, double* gamma = nullptr);
// y = A x in FP32 from the FP16 values of an assembled operator (level 1: K1,
// level 2: A2; ensure_half first)
hipError_t launch_asm_half(const ebe_mesh* m, int level, int nrhs, const float* x, float* y, bool mask_in, bool bc,
                           bool add, const int* gate, hipStream_t s, double* gamma = nullptr);
// FP16 values of an assembled operator from its FP64 values (allocates; synchronous)
ebe_status ensure_half(ebe_mesh* m, int level, hipStream_t s);
// out = bit pattern of max |a_i| (device, one 64-bit word); b = FP16(a * inv_scale)
hipError_t launch_absmax(const double* a, int64_t n, unsigned long long* out, hipStream_t s);
hipError_t launch_to_f16(const double* a, void* b, int64_t n, double inv_scale, hipStream_t s);
hipError_t launch_ebe(const ebe_mesh* m, int order, ebe_dtype dt, int nrhs, const void* x, void* y, bool mask_in,
                      bool bc, bool add, const int* gate, hipStream_t s, double* gamma = nullptr);
// the same with the product form given (0 <= form < EBE_NUM_FORMS)
hipError_t launch_ebe_form(const ebe_mesh* m, int order, int form, ebe_dtype dt, int nrhs, const void* x, void* y,
                           bool mask_in, bool bc, bool add, const int* gate, hipStream_t s, double* gamma = nullptr);
// the form launch_ebe uses for (order, dtype, nrhs)
// form is one of the EBE_FORM_* values and exists at this order (assembled: linear only)
bool form_available(int order, int form);
// ... and it can run on this mesh for (dtype, nrhs): the pipelined and
// coloured forms need the element node words (meshes below 2^25 nodes) and
// node rows addressable with 32-bit byte offsets; the coloured form needs
// the patch colouring
bool form_usable(const ebe_mesh* m, int order, int form, ebe_dtype dt, int nrhs);
int product_form(const ebe_mesh* m, int order, ebe_dtype dt, int nrhs);
// the form and its kernel variant as one key (graph keys: a replay must run the same kernels)
inline uintptr_t product_key(const ebe_mesh* m, int order, ebe_dtype dt, int nrhs) {
  return uintptr_t(product_form(m, order, dt, nrhs)) |
         (uintptr_t(m->fvar[order == 2 ? 0 : 1][dt == EBE_F64 ? 0 : 1][nrhs]) << 8);
}
// time every form of y = K x on this mesh (x, y: device vectors of the
// level's size; y is overwritten) and record the fastest; synchronous.
ebe_status tune_product(ebe_mesh* m, int level, ebe_dtype dt, int nrhs, const void* x, void* y, hipStream_t s,
                        double ms[EBE_NUM_FORMS]);
hipError_t launch_diag_blocks(const ebe_mesh* m, int level, double* blk6, hipStream_t s);
hipError_t launch_invert_blocks(const ebe_mesh* m, int level, const double* blk6, double* inv64,
                                float* inv32, hipStream_t s);
hipError_t launch_expand_blocks(int64_t n, const double* blk6, double* out9, hipStream_t s);
hipError_t launch_lame(const ebe_mesh* m, hipStream_t s);
hipError_t launch_geometry(const ebe_mesh* m, ebe_dtype dt, void* out, hipStream_t s);
// K1 of the linear (corner) mesh into k1.val[0] (FP64, atomics into zeroed
// blocks), and its FP32 copy into k1.val[1] when f32 is set
// assemble: form the FP64 values (zeroed first); f32: copy them to the FP32 values
hipError_t launch_assemble_p1(const ebe_mesh* m, bool assemble, bool f32, hipStream_t s);
// P2 (FP64 and FP32) from the FP64 K1 values and the level-1 block Jacobi,
// then A2 = P2^T K1p P2 (FP64 atomics into zeroed blocks) when assemble is
// set; the FP32 copy of A2 when f32 is set
hipError_t launch_assemble_a2(const ebe_mesh* m, bool assemble, bool f32, hipStream_t s);
// FP64 diagonal blocks of an assembled operator as 6 symmetric values per row
hipError_t launch_asm_diag(const AsmOp& op, double* blk6, hipStream_t s);
hipError_t launch_check_material(const double* young, const double* poisson, int64_t n, int* bad,
                                 hipStream_t s);

// ---- vector kernels (ebe_vec.hip) -----------------------------------------
hipError_t launch_prolong(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y,
                          bool bc, hipStream_t s);
hipError_t launch_restrict(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y,
                           bool bc, hipStream_t s);
// level 2: y[Nv] = P2 x[Na] (zero at fixed DOFs), y[Na] = P2^T x[Nv] (zero at fixed coarse DOFs)
hipError_t launch_prolong_p2(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, hipStream_t s);
hipError_t launch_restrict_p2(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, hipStream_t s);
hipError_t launch_bjacobi(const ebe_mesh* m, int level, ebe_dtype dt, int nrhs, const void* x,
                          void* y, hipStream_t s);

// ---- adjoint (ebe_adjoint.hip) ---------------------------------------------
hipError_t launch_adjoint(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* u,
                          const void* lam, void* g, hipStream_t s);

ebe_status ensure_blocks(ebe_mesh* m, hipStream_t s);
// fill the geometry cache of dtype dt if needed (allocates: call before any
// graph capture; every entry point that launches products does)
ebe_status ensure_geometry(ebe_mesh* m, ebe_dtype dt, hipStream_t s);
// build the assembled linear-level operator of dtype dt if needed (allocates)
ebe_status ensure_assembled(ebe_mesh* m, ebe_dtype dt, hipStream_t s);
// everything products of (level, dtype, nrhs) in their current form need:
// staging, geometry cache, assembled operator (allocates: before any capture)
ebe_status prepare_products(ebe_mesh* m, int level, ebe_dtype dt, int nrhs, hipStream_t s);
ebe_status build_patches(ebe_mesh* m, const int32_t* conn10, const uint8_t* fix, hipStream_t s);
// ---- assembled operators (assembled.cpp) ------------------------------------
// CSR rows (each increasing, non-empty) -> sliced layout with the columns' fix bits
ebe_status slice_rows(const std::vector<int32_t>& ptr, const std::vector<int32_t>& col, const uint8_t* fix,
                      std::vector<int32_t>& soff, std::vector<int32_t>& scol);
ebe_status upload_asm(AsmOp& op, int64_t rows, const std::vector<int32_t>& soff, const std::vector<int32_t>& scol,
                      hipStream_t s);
// aggregation, coarse fix bits, the structures of P2, P2^T and A2
ebe_status build_level2(ebe_mesh* m, const std::vector<int32_t>& bptr, const std::vector<int32_t>& bcol,
                        const uint8_t* fix, hipStream_t s);
// A2 values (FP64, and FP32 when asked) and the level-2 block Jacobi (allocates)
ebe_status ensure_level2(ebe_mesh* m, ebe_dtype dt, hipStream_t s);
// grow the staging buffers for products with up to nrhs cases of the given element size
ebe_status ensure_stage(ebe_mesh* m, int nrhs, size_t elem_bytes);

// ---- deterministic product form (ebe_det.hip) -------------------------------
// y = K x (quadratic level) with no atomics in the sums; needs the geometry
// cache of dtype dt and the staging buffer (prepare_products).  colour: the
// patches colour by colour with sums straight into y (else staging and the
// shared-node pass)
hipError_t launch_det(const ebe_mesh* m, ebe_dtype dt, int nrhs, bool colour, const void* x, void* y, bool mask_in,
                      bool bc, bool add, const int* gate, hipStream_t s, double* gamma);

// ---- allocation-free product (ebe_kernels.hip) ------------------------------
// Size of the fixed device array that stages shared-node partial sums for
// ebe_matvec_noalloc (nslots * 3 * nrhs values of the dtype must fit).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
// device address of that array on `device` (looked up once per device)
ebe_status noalloc_scratch(int device, void** ptr);
// y = K x (or P K P x) in the gather form with the staging in `stage` (the
// scratch array's device address); geometry from the mesh's cache when it
// exists, else from the corner coordinates; allocates nothing
hipError_t launch_ebe_noalloc(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, bool bc,
                              void* stage, hipStream_t s);

}  // namespace ebe
