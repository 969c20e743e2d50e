// FP64 factorisations used by the MPS compression sweeps:
// blocked Householder QR and one-sided Jacobi SVD with an on-device rank rule.
#pragma once
#include <atomic>
#include <vector>

#include "arena.hpp"
#include "common.hpp"

namespace mpsv {

// One block of Householder reflectors acting on rows [k0, m) of the
// factored matrix.  Register-resident panels (reg) keep the reflectors
// column-major, V[j*(m-k0) + i], with their tau; the LDS panels keep the
// compact-WY form H = I - V T V^T with V (m-k0) x jb row-major and Y = V T.
// One panel of a blocked QR: either a register panel (reflectors V, tau
// over the rows from k0 on) or, for blocks taller than 2048 rows, a TSQR
// panel: chunks of crows rows with their own reflectors (V at c*crows*jb,
// tau at c*jb) and the reflectors Vt, taut of the stacked chunk factors
// (srows rows, chunk c's at rows c*jb).
// A group (grp > 0, the compact-WY mode on blocks over 512 rows) is grp
// register panels of 16 columns whose jb reflectors act as one block: V in
// the storage of qr_wy_group_apply, tau in order and its T (64 x 64).
struct QrPanel {
  int k0 = 0, jb = 0;
  bool reg = false;
  int grp = 0;
  double* T = nullptr;
  double* V = nullptr;
  double* tau = nullptr;
  int crows = 0, srows = 0;
  double* Vt = nullptr;
  double* taut = nullptr;
};

struct QrFactor {
  int m = 0, n = 0, k = 0;
  std::vector<QrPanel> panels;
};

// In-place QR of the row-major m x n matrix A (leading dimension ld):
// `f` describes Q = H_0 H_1 ... H_{k-1} (reflector storage from `ws`).  R
// (k = min(m, n) rows, zeros below the diagonal) goes to the view R when
// given (then A itself may be left unchanged), else to the upper trapezoid
// of A.
void qr_factor(hipStream_t s, Arena& ws, double* A, int m, int n, long ld,
               QrFactor& f, MatView R = MatView{nullptr, 0, 0, 0});

// QR of a read-only strided m x n matrix (a transpose, say); R to the view R.
void qr_factor_view(hipStream_t s, Arena& ws, CMatView A, int m, int n,
                    QrFactor& f, MatView R);

// X (m x nc, row-major, leading dimension ldx) <- Q X.
void qr_apply_q(hipStream_t s, Arena& ws, const QrFactor& f, double* X,
                int nc, long ldx);

// Yout (f.m x nc) <- Q [Yin rows 0 .. rows_in-1; 0]; views with any strides
// when Q is one register panel, row-major Yout otherwise.  Yout may alias
// Yin with the same strides.
void qr_apply_q_view(hipStream_t s, Arena& ws, const QrFactor& f, CMatView Yin,
                     int rows_in, MatView Yout, int nc);

// Copy the k x n upper trapezoid of A (zeros below the diagonal) to R.
void extract_r(hipStream_t s, const double* A, int k, int n, long ld,
               MatView R);

// out (rows x cols) <- in for rows < rows_in, 0 below; any strides.
// Gather (gather = true) the chunk-top rows of a TSQR panel from X into T
// (srows x nc, row-major), or scatter T back: stacked row t is row
// (t / jb) * crows + t % jb of X (leading dimension ld).
void chunk_tops(hipStream_t s, double* X, long ld, int crows, int jb, int srows,
                int nc, double* T, bool gather);

void copy_view(hipStream_t s, CMatView in, int rows_in, MatView out, int rows,
               int cols);

// Outcome words of the truncated SVDs of one lane (a stream driven by one
// host thread), owned by whoever drives the lane (an engine keeps one per
// stream it uses).  Each SVD's kernels write kInfoWords doubles of device
// memory: [0] kept rank D, [1] relative discarded weight, [2] sweeps, [3]
// converged, [4] rotation steps, [5] 1 if split workgroups failed to meet.
//
// Between begin() and end(), fixed-rank SVDs (tol <= 0, whose rank the host
// knows in advance) write into a slot of the device ring instead of being
// read back one by one, so the host never waits inside a compression sweep;
// end() synchronises the stream, copies the used slots of every lock-step
// instance back, checks convergence and the rendezvous of each, writes the
// discarded weights to their host destinations and throws the first
// failure.  cancel() synchronises and drops the record (error paths).
// take()/resume() keep a closed record across the replays of a captured
// graph, which write the same slots.
class SvdOutcomes {
 public:
  static constexpr int kSlots = 4096;
  static constexpr int kInfoWords = 8;
  // ring: device, kSlots * kInfoWords doubles (per instance)
  void bind(double* ring) { ring_ = ring; }
  bool bound() const { return ring_ != nullptr; }
  void begin();
  void end(hipStream_t s);
  void cancel(hipStream_t s) noexcept;
  bool deferring() const { return on_ && rec_.used < kSlots; }
  // reserves the next slot: its device words; the discarded weight goes to
  // disc + i * disc_stride for instance i (disc may be null)
  double* reserve(double* disc, long disc_stride, bool split);

  struct Record {
    int used = 0;
    std::vector<std::pair<double*, int>> disc;
    std::vector<long> disc_stride;
    std::vector<char> split;
  };
  Record take();
  void resume(const Record& r);
  // page-locked host words for a read-back on this lane (shared with end())
  double* host_words(size_t n) { return (double*)host_.get(n * sizeof(double)); }

 private:
  double* ring_ = nullptr;
  bool on_ = false;
  Record rec_;
  PinnedBuf host_;  // the read-back of every instance's used slots
};

// Truncated SVD of the row-major m x c matrix X (leading dimension ldx).
// Keeps D = min(cap, rank rule(tol)) singular triplets, D >= 1.
// Outputs (device, row-major):
//   Vt  : D x c,   rows = right singular vectors of the kept values
//   US  : m x D,   columns = u_i * sigma_i (leading dimension ldus = D)
//   sig : (optional, length >= min(m,c)) all singular values, descending
// Returns D and the relative discarded weight sqrt(sum_{i>D} s_i^2 /
// sum s_i^2) in *discarded.  X is overwritten.  With `out` deferring and
// tol <= 0 the call returns without synchronising: D is then min(cap, m,
// c) whatever the values and the discarded weight (disc_stride apart for
// lock-step instances) is written when the deferred section ends.
// Otherwise the stream is synchronised to read D back (one instance only).
int svd_truncate(hipStream_t s, Arena& ws, double* X, int m, int c, long ldx,
                 int cap, double tol, double* Vt, double* US, double* sig,
                 double* discarded, SvdOutcomes* out = nullptr,
                 long disc_stride = 0);

// Device-side counters of the last factorisations (for diagnostics/tests).
struct LinalgStats {
  std::atomic<long> qr_calls{0}, svd_calls{0}, jacobi_sweeps{0};
};
LinalgStats& linalg_stats();

// Maximum Jacobi sweeps (tests lower it to force a convergence failure).
void set_jacobi_max_sweeps(int n);
int jacobi_max_sweeps();

}  // namespace mpsv
