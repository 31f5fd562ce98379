// Internal declarations shared by the HIP translation units of libpdmk.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <array>
#include <vector>

#include "../../include/pdmk.h"
#include "planner.h"

struct pdmk_plan;

namespace pdmk {
struct BoundState;

// ---------------------------------------------------------------- errors
struct Error {
  int code;
  std::string msg;
};
#define PDMK_HIP(call)                                                          \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess)                                                       \
      throw ::pdmk::Error{e_ == hipErrorOutOfMemory ? PDMK_ERR_OUT_OF_MEMORY    \
                                                    : PDMK_ERR_HIP,             \
                          std::string(#call) + ": " + hipGetErrorString(e_)};   \
  } while (0)

// Workspace of one evaluation: a bump allocator over the plan's arena (one
// device buffer kept between calls).  Requests beyond the arena get their own
// hipMalloc for this call; the plan then grows the arena to the call's total
// so that later calls of the same size allocate nothing.
struct Workspace {
  char* base = nullptr;      // plan arena
  size_t size = 0;           // arena bytes
  size_t used = 0;           // bytes handed out this call (arena + overflow)
  bool fixed = false;        // no allocation: a request past `size` is an error
  std::vector<void*> overflow;
  void* take(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (used + bytes <= size) {
      p = base + used;
    } else if (fixed) {
      throw ::pdmk::Error{PDMK_ERR_SCRATCH,
                          "the input needs more than the " + std::to_string(size >> 20) +
                              " MiB of device scratch of the allocation-free entry point"};
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess)
        throw ::pdmk::Error{e == hipErrorOutOfMemory ? PDMK_ERR_OUT_OF_MEMORY : PDMK_ERR_HIP,
                            std::string("hipMalloc: ") + hipGetErrorString(e)};
      overflow.push_back(p);
    }
    used += bytes;
    return p;
  }
  // Call after the stream has drained.
  void release_overflow() {
    for (void* p : overflow) (void)hipFree(p);
    overflow.clear();
  }
};

// Smallest eps at which a mixed plan computes stages in FP32.
constexpr double kMixedEpsFloor = 1e-6;

// Zeroes `bytes` bytes at p with a fill kernel on stream s (used instead of
// hipMemsetAsync on every path a caller may capture into a HIP graph).
void fill_zero(void* p, size_t bytes, hipStream_t s);

// Raises a kernel's dynamic-LDS limit (per device) to at least `bytes`.  The
// limit only grows, under a process-wide lock, so a thread evaluating one
// plan never lowers the limit another thread's launch relies on.
void ensure_lds(const void* kernel, size_t bytes);

// Largest number of sources plus images (sorted indices, tree ranges and
// list entries are int32).
constexpr int64_t kMaxImages = ((int64_t)1 << 31) - 4096;

// Sources per work item of the leaf residual sums: a target leaf's source
// list is cut into segments of this length, so that the cost of one block is
// bounded by kDirectTgt x kDirectSeg pairs.
constexpr int kDirectSeg = 4096;
// Targets per work item of the leaf residual sums (one 64-lane pass).
constexpr int kDirectTgt = 64;

// ------------------------------------------------------- device constants
// Everything a kernel needs about the method, passed by value.
struct KParams {
  int dim;
  int p;            // proxy points per axis
  int J;            // plane-wave half count
  int nE, nF2;      // series lengths (FP64 evaluation)
  int nEd, nF2d;
  int nE32, nF232;  // series lengths for FP32 evaluation (cut at FP32 resolution)
  int nEd32, nF2d32;
  int B;            // Morton bits per axis
  int next[3];      // extended root grid dims
  double rc;
  double irc;   // 1 / rc
  double origin[3];
  double L[9], Li[9], Q[9];
  double w0unit;    // W_h(0) for h = 1
  int precision;
  int bloch;        // quasi-periodic conditions (Section 4.1)
  double beta[3];   // Bloch vector in the oriented frame
  int vimg;         // images as virtual neighbours (rem:cube)
};

// Lattice shift of a colleague or list entry under virtual images: code
// 1 + sum_a (n_a + 1) 3^a for n in {-1, 0, 1}^d, 0 for no shift.
__host__ __device__ inline int shift_code(const int* n, int d) {
  int c = 0, m = 1;
  for (int a = 0; a < d; ++a) {
    c += (n[a] + 1) * m;
    m *= 3;
  }
  return c == (d == 3 ? 13 : 4) ? 0 : c + 1;
}

// One tree level (device arrays; counts on host).
struct Level {
  int n = 0;                 // boxes
  uint64_t* key = nullptr;   // smallest point key in the box
  int* coord = nullptr;      // dim ints per box
  int* sbeg = nullptr;       // source range in sorted sources
  int* send = nullptr;
  int* tbeg = nullptr;       // target range in sorted targets
  int* tend = nullptr;
  int* parent = nullptr;
  int* child0 = nullptr;     // first of 2^d children at the next level, -1 = leaf
  int* coll = nullptr;       // 3^d colleague indices, -1 = none
  unsigned char* cshift = nullptr;  // virtual images: shift_code of each colleague
  int* nlid = nullptr;       // index among non-leaf boxes of this level, -1 = leaf
  int nnl = 0;               // non-leaf count
  int* nl_box = nullptr;     // non-leaf index -> box index
  void* proxy_q = nullptr;   // nnl * p^d outgoing proxy charges (FP64 or FP32)
  void* proxy_phi = nullptr; // nnl * p^d incoming proxy potentials
};

// Per-evaluation state.
struct Eval {
  hipStream_t s = nullptr;
  Workspace* ws = nullptr;
  pdmk_plan* plan = nullptr;   // events come from its pool
  hipEvent_t event();
  template <class T>
  T* alloc(size_t n) {
    return static_cast<T*>(ws->take(n * sizeof(T)));
  }
  int64_t n_src = 0, n_trg = 0, n_img = 0;
  bool self_targets = true;
  // sources after orientation and wrap (SoA, FP64)
  double* xs = nullptr;   // dim * n_src
  double* us = nullptr;   // fractional
  double* xt = nullptr;   // targets (== xs when self_targets)
  double* ut = nullptr;
  const double* q = nullptr;
  // sorted sources (originals + images) and sorted targets
  double* sx = nullptr;   // dim * n_img
  double* sq = nullptr;
  uint64_t* skey = nullptr;
  double* tx = nullptr;   // dim * n_trg
  uint64_t* tkey = nullptr;
  int* tperm = nullptr;   // sorted target -> original target index
  double* ox = nullptr;   // original sources in tree order (dim * n_src), for the far field
  double* oq = nullptr;
  // Bloch conditions: wrap phases of sources and targets (beta.L w), the
  // imaginary parts of the wrapped charges (unsorted; q holds the real
  // parts), of the sorted image charges and of the originals in tree order
  double* theta_s = nullptr;
  double* theta_t = nullptr;
  const double* q_im = nullptr;
  double* sq_im = nullptr;
  double* oq_im = nullptr;
  // kept-tree evaluation (pdmk_plan_bind / pdmk_plan_execute)
  bool keep_map = false;    // stage_images also writes img_src (and operm)
  int* img_src = nullptr;   // sorted image -> source index
  int* operm = nullptr;     // separate targets: ox / oq entry -> source index (else null:
                            // ox is tx and oq follows tperm)
  bool timing = true;       // record per-stage events (off inside pdmk_plan_execute)
  bool det = false;         // PDMK_DETERMINISTIC
  // residual pairs evaluated once (targets = sources): the lists of a leaf
  // skip all-real boxes whose sources precede its own, and the residual sums
  // add each pair to both ends.  img_trg: sorted image -> sorted target index
  // of the point it is (-1 for a shifted copy)
  bool sym = false;
  int* img_trg = nullptr;
  std::vector<Level> lev;
  Level* d_lev = nullptr;   // device copy of lev (for list building)
  // target leaves
  int nleaf_t = 0;          // list slots: every box of every level
  int* lf_box = nullptr;    // (level << 26 | box) packed as two arrays
  int* lf_level = nullptr;
  int* lf_boxid = nullptr;
  int* lf_list_beg = nullptr;
  int4* list = nullptr;     // {sbeg, send, level, 0}
  int64_t nlist = 0;
  int* lf_nsrc = nullptr;   // sources in each target leaf's list
  int2* items = nullptr;    // residual-sum work items (leaf, segment), heaviest first
  int2* items_u = nullptr;  // the same in list order: item_beg[leaf] + segment
  int* item_beg = nullptr;  // first work item of each list slot (list order)
  int nitems = 0;
  double* pot_sorted = nullptr;   // near field per sorted target
  double* grad_sorted = nullptr;
  pdmk_stats st{};
  // near-field timing and counters, read once the call's stream has finished
  // (no host wait inside the pipeline): events e0..e3 around residual sums,
  // plane waves, leaf evaluation; per level {start, outgoing done, incoming
  // done, translation done}; device counters copied into the plan's pinned
  // host buffer
  int* d_flags = nullptr;   // device {non-finite charge, non-finite position}
  double* qsum = nullptr;   // device {sum q, sum |q|}
  bool near_pending = false;
  // the axis-by-axis plane waves may call the library GEMM (it may allocate:
  // not in the allocation-free entry or a kept-tree execute)
  bool lib_gemm = false;
  double* far_out = nullptr;    // separate far-field part (tree order), else null:
                                // the interpolation adds into pot_sorted
  int far_comp = 0;             // grid part the interpolation reads (1: imaginary)
  double* far_grid = nullptr;   // spreading grid (real)
  unsigned long long* far_hi = nullptr;   // fixed-order mode: fixed-point grid words
  unsigned long long* far_lo = nullptr;
  double2* far_cg = nullptr;    // its transform, scaled and transformed back
  bool pw_split = false;
  hipEvent_t near_ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // far field: spreading start / end, transforms end, interpolation start / end
  hipEvent_t far_ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  std::vector<std::array<hipEvent_t, 4>> pw_ev;
};
// Fills the near-field entries of E.st (call after the stream has finished).
void near_finish(const pdmk_plan* P, Eval& E);
// Colleague translation of one level on compact half-ball expansions (3D, FP64).
void pw_translate(const pdmk_plan* P, const Level& L, const double2* S, double2* Iw,
                  double levfac, unsigned long long* npairs, hipStream_t s);
// Destroys the plan's library-GEMM handle (if one was made).
void gemm_release(pdmk_plan* P);

}  // namespace pdmk

// The plan (C-ABI opaque type).
struct pdmk_plan {
  pdmk_opts o{};
  pdmk::MethodParams mp{};
  pdmk::Geometry g;
  const pdmk::SplitTables* T = nullptr;
  const pdmk::Pswf* P = nullptr;
  int device = 0;
  char* arena = nullptr;        // device workspace kept between calls
  size_t arena_size = 0;
  // real matrices of the plane-wave contractions for the matrix-core path
  float* d_pwt_f = nullptr;
  double* d_pwt_d = nullptr;
  float* d_pwt_b = nullptr;     // FP32 values, depths padded for the BF16 products
  size_t pwt_off[6] = {0, 0, 0, 0, 0, 0};
  size_t pwt_off_b[6] = {0, 0, 0, 0, 0, 0};
  int* d_ball = nullptr;        // modes of the half ball, then the slab starts
  int2* d_brow = nullptr;       // per mode row (j0, j1 + J): {index of j2 = -J, half width}
  int nball = 0;
  bool pw_mfma = true;          // use the matrix-core plane-wave kernels when they fit
  // stages that run in FP32 in mixed mode: 1 residual sums, 2 proxies and
  // plane waves, 4 far-field window weights; 8: BF16 plane-wave products at
  // eps >= 1e-3 (all by default)
  unsigned mixed_parts = 15;
  // HIP events reused by every call on this plan (created on first use;
  // a plan serves one call at a time)
  std::vector<hipEvent_t> ev_pool;
  size_t ev_next = 0;
  double* adj_buf = nullptr;    // Psi and grad Psi of the adjoint (n_src (d + 1))
  // pinned host: [0..2] plane-wave pairs, boxes, support pairs; [3] visited
  // residual pairs; [4..5] sum q,
  // sum |q| (FP64 bits); [6] the two input flags of Eval::d_flags; [8] residual
  // pairs staged after the per-pass reach test
  unsigned long long* h_cnt = nullptr;
  // second stream (default priority, created on first use): the far field's
  // grid steps run on it beside the tree, list and near-field stages
  hipStream_t s_aux = nullptr;
  size_t adj_size = 0;
  pdmk::KParams kp{};
  // device tables
  // residual series as monomials in u = 2 s - 1 (s = r^2 / h^2): entries
  // [0, 32) for FP64 evaluation, [32, 64) cut for FP32 evaluation
  double* d_E = nullptr;
  double* d_Ed = nullptr;       // dE/ds
  double* d_F2d = nullptr;      // dF2/ds
  double* d_F2 = nullptr;
  double* d_nodes = nullptr;   // p
  double* d_bw = nullptr;      // p
  double* d_Tm = nullptr;      // [2][p][p]: parent basis at child nodes, sigma = -1, +1
  double2* d_F = nullptr;      // [2J+1][p]: exp(-i pi j xi_p / 3)
  double2* d_Fc = nullptr;     // its conjugate
  double2* d_Fw = nullptr;     // its conjugate with rows j > 0 doubled (Hermitian half)
  void* blas = nullptr;        // rocBLAS handle of the library-GEMM plane-wave path
  float2* d_Ff = nullptr;      // FP32 copy
  double* d_dtab = nullptr;    // |j|^2 table
  double* d_farscale = nullptr;// M0*M1*M2
  double2* d_fftw = nullptr;   // FFT twiddles exp(-2 pi i k / M_a) per axis
  int64_t fftw_off[3] = {0, 0, 0};
  double* d_shiftvec = nullptr;  // nshift * dim lattice translations L n
  int nshift = 0;
  double nufft_beta = 0;
  pdmk_stats last{};
  pdmk::BoundState* bound = nullptr;   // tree kept by pdmk_plan_bind
};

namespace pdmk {
inline hipEvent_t Eval::event() {
  pdmk_plan* P = plan;
  if (P->ev_next < P->ev_pool.size()) return P->ev_pool[P->ev_next++];
  hipEvent_t e = nullptr;
  PDMK_HIP(hipEventCreate(&e));
  P->ev_pool.push_back(e);
  ++P->ev_next;
  return e;
}

// Matrix-core plane-wave transforms (pwmfma.hip).
constexpr int kPwMaxTiles = 16;   // accumulator tiles of a box's proxy potential per wave
struct PwMfmaShape {
  bool ok;
  int g_out, g_in;              // slabs j0 per group
  size_t lds_out, lds_in;       // dynamic LDS bytes
  int sX, sZ, sI, sY, sW;       // LDS row strides
};
// kb: k-steps of 4 per product (1: FP32 / FP64 16x16x4; 4: BF16 16x16x16)
PwMfmaShape pw_mfma_shape(int p, int J, size_t real_size, int kb = 1);
void pw_mfma_upload(pdmk_plan* P);
// One level: outgoing expansions into S (compact half-ball order), the
// colleague translation into Iw, incoming expansions into proxy_phi; ev_out /
// ev_tr (optional) are recorded after the first two kernels.
template <class Real>
void pw_mfma_level(const pdmk_plan* P, const Level& L, int nn, const void* proxy_q, void* S,
                   void* Iw, void* proxy_phi, double levfac, unsigned long long* npairs,
                   hipEvent_t ev_out, hipEvent_t ev_tr, hipStream_t s);

template <class Real>
bool eval_leaf_mfma(const pdmk_plan* P, const Level& Lp, const Level& Lc, int l,
                    const double* tx, int64_t ntrg, double* pot, double* grad, hipStream_t s);

template <class Real>
bool anterp_mfma(const pdmk_plan* P, const Level& L, const Level& C, int l, const double* sx,
                 const double* sq, int64_t nimg, void* Q, hipStream_t s);

// det: children add into their parents one octant per launch (fixed order)
template <class Real>
bool transfer_mfma(const pdmk_plan* P, const Level& Lp, const Level& Lc, bool up,
                   const void* src, void* dst, bool det, hipStream_t s);

// stages (implemented in tree.hip / near.hip / far.hip)
void stage_prepare(pdmk_plan* P, Eval& E, const double* src, const double* trg);
void stage_images(pdmk_plan* P, Eval& E, const double* q);
void stage_tree(pdmk_plan* P, Eval& E);
void stage_lists(pdmk_plan* P, Eval& E);
void stage_near(pdmk_plan* P, Eval& E, bool want_grad);
// far field, steps one to four (spreading, transforms, scaling) on E.s, and
// step five (interpolation, adds into pot_sorted) on E.s
void stage_far_grid(pdmk_plan* P, Eval& E);
void stage_far_interp(pdmk_plan* P, Eval& E, bool want_grad);
void stage_assemble(pdmk_plan* P, Eval& E, const double* q, double* pot, double* grad);
void plan_upload_tables(pdmk_plan* P);
void far_build_scale(pdmk_plan* P);

// scans (rocprim)
void exclusive_scan_int(const int* in, int* out, int n, Eval& E);
int read_int(const int* dptr, hipStream_t s);
}  // namespace pdmk
