// Internal declarations shared by the host sources of libhgrape.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hgrape.h"

namespace hg {

constexpr int kMaxDiag = 16;      // storage for the union diagonals (DIA width)
constexpr int kMaxDiagKernels = 13;  // widest union pattern the sweep kernels are built for
constexpr int kMaxDiagCtrl = 4;   // diagonals of one control operator
constexpr int kMaxCtrl = 16;      // control channels
constexpr int kMaxThreads = 512;  // threads per workgroup (2 waves per SIMD)
constexpr int kWideThreads = 1024;   // complex64 workgroups for 512 < d <= 2048 (4 waves per SIMD)
constexpr int kMaxRows = 8;       // rows per thread
constexpr int kMMax = 60;         // largest Taylor degree the planner may choose
constexpr int kSMax = 4096;       // largest scaling factor one step may use

void set_error(const std::string& msg);

// Operators on the device in diagonal (DIA) storage.  Row i of diagonal e
// holds the entry (i, i + off[e]), zero where that column is outside the matrix.
struct DevOps {
  int W = 0;                       // number of union diagonals
  int npure = 0;                   // leading union diagonals on which H_0 and every H_k are real
  // Every control real (ecl 0: E_k = -i (dt/s) e_k) or purely imaginary (ecl 1:
  // E_k = (dt/s) e_k), e_k real: the backward can then carry X_k rotated to
  // the frame where its source E_k Y has real coefficients.
  bool ereal = false;
  int ecl[kMaxCtrl] = {0};
  int off[kMaxDiag] = {0};
  int WK[kMaxCtrl] = {0};          // diagonals per control
  int offk[kMaxCtrl][kMaxDiagCtrl] = {{0}};
  int halo = 0;                    // max |off|: LDS halo on each side of a vector
  double2* vals = nullptr;         // [(K+1)][W][dim]: H0 then H_1..H_K on the union pattern
  double2* valk = nullptr;         // [K][kMaxDiagCtrl][dim]: each H_k on its own diagonals
  double* omega = nullptr;         // [dim] or nullptr
  // Row-indexed (ELL) storage, for patterns that are not a few diagonals:
  // slot e of row i holds the column cols[e][i] (slot 0 the main diagonal,
  // or an all-zero stand-in), control k's entry qq the column colk[k][qq][i];
  // vals/valk are then indexed by slot instead of diagonal, off/offk unused.
  bool ell = false;
  int32_t* cols = nullptr;         // [W][dim]
  int32_t* colk = nullptr;         // [K][kMaxDiagCtrl][dim]
};

constexpr int kDenseMaxDim = 8192;  // dense storage: (K+1) dp^2 complex128 on the device

// A state column too long for one workgroup, split over P co-resident
// workgroups.  The rows are blocks of L (row r = t L + c, t < T): every union
// offset is either a multiple of L (it keeps c) or at most h in size and stays
// inside its block.  Part p owns c in [c0[p], c0[p] + w[p]) of every block, so
// only the h rows at each edge of its c-range couple to a neighbouring part.
// Locally a part stores, per block t, a segment of `seg` rows: h halo rows
// (copies of the left neighbour's edge), its own w[p] rows, h halo rows (the
// right neighbour's edge) and padding; local offsets map q L -> q seg.  The
// local operators are DIA arrays over the T * seg local rows whose halo and
// padding rows are zero, so a part runs the ordinary sweep kernels on them and
// refreshes its halo rows from its neighbours after every Taylor term.
constexpr int kMaxParts = 16;
constexpr int kMaxDimSplit = 65536;
struct Split {
  int P = 1;                      // 1: no split
  int L = 0, T = 0, h = 0, seg = 0, d_loc = 0;
  int w[kMaxParts] = {0}, c0[kMaxParts] = {0};
  DevOps ops;                     // local operators: arrays hold P parts back to back
  size_t vals_stride = 0, valk_stride = 0, omega_stride = 0;  // elements per part
};

// Operators on the device as dense matrices (problems created with dense
// storage): H[o][i][j], o = 0 (H0) then 1..K, row-major, dp = dim rounded up to
// 64, zero outside dim x dim.
struct DenseOps {
  double2* H = nullptr;
  double* omega = nullptr;  // [dim] or nullptr (the problem's penalty diagonal)
};

}  // namespace hg

struct hg_ctx {
  int device = 0;
  int num_cu = 0;
  size_t lds_per_block = 0;
};

struct hg_problem {
  hg_ctx* ctx = nullptr;
  int64_t dim = 0;
  int32_t n_ctrl = 0;
  int32_t sigma = 0;               // max non-zeros in a row of the union pattern
  int64_t nnz = 0;                 // stored union non-zeros (structural)
  std::vector<int64_t> nnz_ctrl;   // structural non-zeros of each H_k
  hg::DevOps ops;
  bool dense = false;              // dense storage: the MFMA path runs, not the DIA kernels
  int64_t dp = 0;                  // padded dimension of the dense matrices
  hg::DenseOps dops;
  hg::Split split;                 // column split for dimensions beyond one workgroup
  ~hg_problem();                   // frees the device arrays (also on a failed creation)
};

namespace hg {

// Planner (plan.cpp): FP64, no contraction, the same operation order as the
// bound of App. C.
double error_bound(double theta, int m, int s, int sigma, double u);
// Returns 0 on success, 1 if unreachable, 2 if a solution would need s > 4096
// (then *fail_index is the failing index).  With build_table, the threshold
// table of (sigma, tau, u) is built and cached on first use (host memory);
// without, a cached table is used as far as it reaches and the direct search
// decides the rest (the same decisions, no allocation).  rule: HG_PLAN_SMALLEST_S
// (the paper's) or HG_PLAN_MIN_MU (fewest products under the same bound).
int plan_steps(const double* theta, int64_t n, int sigma, double tau, double u,
               int32_t* m_out, int32_t* s_out, int64_t* fail_index, bool build_table = true,
               int rule = 0);

// One evaluation (hg_eval's work) on caller-provided memory: `ws` device
// workspace of ws_bytes, `hbuf` host staging of hbuf_bytes (pinned or not).
// OUT_OF_MEMORY when either is too small for the shape.  See plan_steps for
// build_table.
hg_status eval_on_buffers(hg_problem* p, const hg_eval_desc* d, hg_result* results, double* grad,
                          hipStream_t hs, void* ws, size_t ws_bytes, void* hbuf,
                          size_t hbuf_bytes, bool build_table);

// Looks up (once per device, with that device current) the device address of
// hg_eval_noalloc's scratch array (noalloc.cpp).
hg_status noalloc_setup(int device);

// Kernel launchers (kernels.hip).
struct SweepShape {
  int dim, n_ctrl, n_steps, n_states, n_batch;
  int rows_per_thread, threads, groups;  // backward launch; groups = controls per backward pass
  int fwd_rows_per_thread, fwd_threads;  // the forward kernel's own launch shape
  int fwd_cpw;                           // state columns per forward workgroup (1 or 2)
  size_t lds_fwd2;                       // forward LDS with two columns (0: not offered)
  size_t lds_fwd, lds_bwd;
  bool c128;
  int parts;                             // workgroups per state column (1 = no split)
  int spread;                            // backward workgroups sharing a column's controls
  int pure;                              // leading diagonals taken as purely imaginary in B (1 or 3)
  bool ereal;                            // auxiliary vectors in the frame of real E_k (DevOps::ereal)
};
hipError_t launch_step_norms(const DevOps& ops, int dim, int K, const double* u, int nb,
                             int N, double dt, double* theta, hipStream_t st);
hipError_t launch_state_norms(const double* psi, int dim, int S, int nb, double* out,
                              hipStream_t st);

struct SweepBuffers {
  const double* u;
  const int32_t* m_sched;          // [B][N]
  const int32_t* s_sched;          // [B][N]
  const double* psi0;              // [B][S][dim] complex128
  const double* targets;           // [B][S][dim] complex128
  void* psiN;                      // [B][S][dim] working precision
  void* cold;                      // [B][S][Q][3][dim] complex FP64 (carried vectors)
  void* ckpt;                      // checkpoint variant: [B][S][ceil(N/C)][dim], else null
  void* segbuf;                    // checkpoint variant: [B][S][C][dim], else null
  double* ovl;                     // [B][S][2]
  double* ovt;                     // [B][S][N][2] overlaps after every step, or null (w_int == 0)
  double* gt;                      // [B][N][2] their averages over the S states (with ovt)
  double* pen;                     // [B][S]
  double* gradp;                   // [B][S][K][N]
  double* drift;                   // [B][S]
  double* res;                     // [B][8]
  double* grad;                    // [B][K][N] or nullptr
  hipEvent_t ev[3];                // optional: before forward, between, after backward
};
struct SweepParams {
  double dt, w_fid, w_pen, w_int;
  int renorm_every;
  int ckpt_every;  // 0: reconstruction; > 0: checkpoint every C steps
};
bool sweep_supported(const DevOps& ops, int dim, int K, bool c128, size_t lds_limit,
                     SweepShape* shape, std::string* why);
hipError_t launch_sweep(const DevOps& ops, const SweepShape& sh, const SweepBuffers& b,
                        const SweepParams& p, hipStream_t st);

// Split-column sweeps (see Split).  The launch shape of one part's local
// problem, or false with the reason; the sweep itself with split buffers.
bool split_supported(const Split& sp, int K, bool c128, size_t lds_limit, int num_cu,
                     SweepShape* shape, std::string* why);
struct SplitBuffers {
  double2* psi0_loc;               // [B][S*P][d_loc] gathered initial states (zero halo)
  double2* tgt_loc;                // [B][S*P][d_loc] gathered targets
  unsigned char* xbuf;             // exchange rows: [B][S*P][2][2][T h][64 bytes]
  double* xnrm;                    // [B][S*P][kMaxParts] partial norms (ring)
  uint32_t* xflag;                 // [B][S*P] exchange sequence numbers
  uint32_t* xerr;                  // [1] set when a wait timed out
};
hipError_t launch_split_sweep(const Split& sp, const SweepShape& sh, const SweepBuffers& b,
                              const SplitBuffers& x, const SweepParams& p, int S_true,
                              hipStream_t st);

// Dense path (dense_kernels.hip).
struct DenseShape {
  int d, dp, K, N, S, Sp, B;  // Sp = S rounded up to 64
  bool c128;
  int num_cu;                 // compute units of the device (tile choice)
};
struct DenseBuffers {
  const double* u;
  const int32_t* m_sched;          // [B][N]
  const int32_t* s_sched;          // [B][N]
  const double* psi0;              // [B][S][dim] complex128
  const double* targets;           // [B][S][dim] complex128
  void* blocks;                    // dense_block_elems(shape) working-precision reals
  void* mat;                       // [B][2dp][2dp] embedded A_n/s_n
  void* emat;                      // [B][K][2dp][2dp] embedded E_k/s_n
  void* ckpt;                      // checkpoint variant: [B][ceil(N/C)] state groups, else null
  void* segbuf;                    // checkpoint variant: [B][C] state groups, else null
  double* pen;                     // [B][S]
  double* ovl;                     // [B][S][2]
  double* ovt;                     // [B][S][N][2] or null (w_int == 0)
  double* gt;                      // [B][N][2] (with ovt)
  double* drift;                   // [B][S]
  double* res;                     // [B][8]
  double* grad;                    // [B][K][N] or nullptr (then no derivative sweep)
  hipEvent_t ev[3];
};
size_t dense_block_elems(const DenseShape& sh);

// Matrix-diagonalisation variant for dense operators (diag.hip, App. F).
struct DiagBuffers {
  const double* u;
  const double* psi0;              // [B][S][dim] complex128
  const double* targets;           // [B][S][dim] complex128
  void* work;                      // diag_work_bytes(shape)
  int* h_done;                     // host [B]: convergence flags of the eigensolver
  double* pen;                     // [B][S]
  double* ovl;                     // [B][S][2]
  double* ovt;                     // [B][S][N][2] or null (w_int == 0)
  double* gt;                      // [B][N][2] (with ovt)
  double* drift;                   // [B][S]
  double* res;                     // [B][8]
  double* grad;                    // [B][K][N] or nullptr
  hipEvent_t ev[3];
};
size_t diag_work_bytes(const DenseShape& sh);
hipError_t launch_diag_sweep(int dev, const DenseOps& ops, const DenseShape& sh,
                             const DiagBuffers& bf, const SweepParams& sp, hipStream_t st);
hipError_t launch_dense_norms(const DenseOps& ops, int d, int dp, int K, const double* u, int nb,
                              int N, double dt, double* theta, hipStream_t st);
hipError_t launch_dense_sweep(const DenseOps& ops, const DenseShape& sh, const DenseBuffers& bf,
                              const SweepParams& sp, const int32_t* h_m, const int32_t* h_s,
                              hipStream_t st);

}  // namespace hg
