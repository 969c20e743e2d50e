// MPS engine: device MPS/MPO objects, the compression sweep and the RK4 step.
#pragma once
#include <memory>
#include <vector>

#include "arena.hpp"
#include "common.hpp"
#include "linalg.hpp"

namespace mpsv {

struct Problem {
  int Lx = 6, Lv = 6, order = 0;
  double x_min = 0, x_max = 1, v_min = -1, v_max = 1;
  double qm = -1.0, dt = 0.05;
  int chi_max = 16, level = 1, df_max = 0;
  double tol = 1e-10;
  int precision = 0;
  int x_scheme = 0;  // 0 central, 1 upwind x advection
  double cfl = 0.0;  // > 0: adaptive dt, this fraction of the CFL limit
  int compression = 0;  // 0 sweep, 1 centre-first (sequential orderings)
  double nu = 0.0, nu_v0 = 0.0, nu_vth = 1.0;  // Dougherty collisions
  int coll_model = 0;  // 0 drift / thermal speed from the moments of f, 1 fixed
  int tall_apply = 0;  // tall-block reflector application: 0 one at a time, 1 WY
  int n() const { return Lx + Lv; }
  long Nx() const { return 1L << Lx; }
  long Nv() const { return 1L << Lv; }
  double dx() const { return (x_max - x_min) / (double)Nx(); }
  double dv() const { return (v_max - v_min) / (double)(Nv() - 1); }
};

// Sites of the chain as (0 = x / 1 = v, bit k; k = 0 the coarsest) for the
// orderings of Fig. 3: 0 S1 (x then v, both coarse to fine), 1 IF (x1 v1
// x2 v2 ...), 2 S2 (x fine to coarse, then v), 3 S3 (x, then v fine to
// coarse).
std::vector<std::pair<int, int>> site_list(int Lx, int Lv, int order);

// MPS core A[a][s][b], row-major, a < l, s < 2, b < r.
struct Core {
  double* p = nullptr;
  int l = 1, r = 1;
  long size() const { return (long)l * 2 * r; }
};
using DMps = std::vector<Core>;

// MPO site W[b][o][i][b'] and Wmat[(o,b')][(b,i)] (both device).
struct MpoSite {
  double* W = nullptr;
  double* Wmat = nullptr;
  int wl = 1, wr = 1;
};
using DMpo = std::vector<MpoSite>;

// One site of an implicit chain handed to the compression sweep.
struct VSite {
  enum Kind { kDense, kApply, kSum, kCopy } kind = kDense;
  int l = 1, r = 1;
  Core A;                                    // kDense, kApply
  MpoSite W;                                 // kApply
  std::vector<double> coef;                  // kSum
  std::vector<Core> terms;                   // kSum
  std::vector<int> loff, roff;               // kSum block offsets
  int pos = 1;                               // kSum: 0 first, 1 middle, 2 last
};

// Device-memory model of one instance, for admission control.  Per arena
// (operators, committed state, step, rhs, compression, side rhs, side
// compression) `arena[i]` estimates the peak extent in use from three sizes
// at the bond caps: the state S (sum of the chi-capped cores), the widest
// MPO x MPS site contraction N of the field term (interleaved ordering) and
// the size I of the interleaved initial state built from the x and v
// profiles at full rank.  The coefficients envelope the peaks measured
// over 2^6..2^13 grids, chi 16..128, both orderings and D_F in {4, chi}.
// `chunk` is the arena chunk size; `bound` adds two chunks per arena for
// rounding and a fixed 32 MiB.
struct MemoryModel {
  size_t arena[7];
  size_t chunk, bound;
};
MemoryModel memory_model(const Problem& p);

// Throws Error(kEinval) for a problem the engine does not accept.
void validate_problem(const Problem& p);

struct StepTimers {
  double compress_ms = 0;
};

class Engine;
// several species sharing x and E (see step_species in engine.cpp)
void step_species(const std::vector<Engine*>& es, const std::vector<double>& q,
                  hipStream_t s);
void field_species_dense(const std::vector<Engine*>& es, const std::vector<double>& q,
                         double* E_out, double* energy, hipStream_t s);

// An engine holds one instance, or a batch of lock-step instances of one
// problem shape (see Lanes): the same grid sizes, ordering, caps, level,
// precision, schemes and time step, tol = 0 and a fixed dt, so that every
// compression keeps the same ranks in all of them; their physical
// parameters (intervals, collision constants) and data may differ.  A
// batched step issues each launch once for all instances.
class Engine {
  friend void step_species(const std::vector<Engine*>&, const std::vector<double>&,
                           hipStream_t);
  friend void field_species_dense(const std::vector<Engine*>&,
                                  const std::vector<double>&, double*, double*,
                                  hipStream_t);
  friend DMps field_of_species(const std::vector<Engine*>&, const std::vector<double>&,
                               const std::vector<const DMps*>&, Arena&, hipStream_t);

 public:
  explicit Engine(const Problem& p);
  explicit Engine(const std::vector<Problem>& batch);
  ~Engine();
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;

  const Problem& problem() const { return p_; }
  int n() const { return p_.n(); }
  int instances() const { return nin_; }

  // ---- state (per instance; instance 0 of a batch fixes the bond
  // dimensions that every other instance must then have)
  void init_from_profiles(int rank, const double* ax, const double* bv,
                          hipStream_t s, int inst = 0);
  void set_state(const std::vector<int>& bonds, const double* packed,
                 hipStream_t s, int inst = 0);
  void get_state(std::vector<int>& bonds, double* packed, hipStream_t s,
                 int inst = 0) const;
  void add_scaled(double alpha, const std::vector<int>& bonds,
                  const double* packed, hipStream_t s, int inst = 0);
  // ---- state of every instance of a batch at once
  // each instance's initial state from its profiles (device, rank x N)
  void init_batch(const std::vector<int>& ranks, const std::vector<const double*>& ax,
                  const std::vector<const double*>& bv, hipStream_t s);
  // packed device cores per instance, one set of bonds
  void set_states(const std::vector<int>& bonds, const std::vector<const double*>& packed,
                  hipStream_t s);
  // f_i <- compress(f_i + alpha_i g_i), packed device cores g_i per instance
  void add_scaled_all(const std::vector<double>& alpha, const std::vector<int>& bonds,
                      const std::vector<const double*>& packed, hipStream_t s);
  const DMps& state() const { return f_; }
  std::vector<int> bonds() const;
  double time() const { return t_; }
  // von Neumann entropy (log2) of the Schmidt values at each of the n-1
  // bonds of the committed state (an untruncated canonicalisation)
  std::vector<double> entanglement(hipStream_t s, int inst = 0);
  // the step the next mps_step takes (the adaptive one needs a sync)
  double step_size(hipStream_t s);
  long steps_done() const { return steps_; }
  // relative discarded weight per bond of the last compression of instance
  // inst (n - 1 values)
  std::vector<double> last_discarded(int inst = 0) const;

  // ---- the hot path
  void step(hipStream_t s);
  // Steps of fixed shape (tol = 0, fixed dt) can replay a captured graph of
  // the step's launches: the first step from a state layout runs eagerly
  // (sizing every workspace), the second is recorded on the instance's own
  // stream by one host thread (both lanes) and replayed, later ones replay.
  void set_step_graph(bool on) { graph_on_ = on; }
  long graph_captures() const { return graph_captures_; }
  long graph_replays() const { return graph_replays_; }
  // A stream owned by this instance (batched stepping runs each instance on
  // its own stream).
  hipStream_t own_stream() const { return own_; }
  // device bytes currently held by this state's arenas
  size_t device_bytes() const;
  // per arena (operators, state, step, rhs, compression, side rhs, side
  // compression): reserved bytes and peak extent in use
  void arena_bytes(size_t reserved[7], size_t peak[7]) const;

  // ---- outputs (per instance)
  void to_dense(double* out, hipStream_t s, int inst = 0);
  void moments(double* n_out, double* E_out, double* scalars, hipStream_t s,
               int inst = 0);
  void density_field(double* n_out, double* E_out, hipStream_t s,
                     int inst = 0);

  // ---- building blocks exposed for tests through the C-ABI
  // QR sweep left to right, then truncated SVD sweep right to left; with
  // centre > 0 the centre-first scheme cut at the bond centre-1 | centre
  DMps compress_chain(const std::vector<VSite>& ch, int cap, double tol,
                      Arena& out, hipStream_t s, std::vector<double>* disc,
                      std::vector<std::vector<double>>* sigmas = nullptr,
                      int centre = 0);
  // centre < 0: the problem's scheme (centre-first at the x|v bond for a
  // full chain when the problem asks for it)
  DMps compress_mps(const DMps& a, int cap, double tol, Arena& out,
                    hipStream_t s, std::vector<double>* disc = nullptr,
                    int centre = -1);
  DMps apply_compress(const DMpo& W, const DMps& a, int cap, double tol,
                      Arena& out, hipStream_t s,
                      std::vector<double>* disc = nullptr);
  DMpo upload_mpo(const std::vector<std::vector<double>>& W,
                  const std::vector<int>& bonds, Arena& ar, hipStream_t s);
  // one host MPO per instance of the calling thread's lanes
  DMpo upload_mpo(const std::vector<const std::vector<std::vector<double>>*>& Ws,
                  const std::vector<int>& bonds, Arena& ar, hipStream_t s);

  DMps add_terms(const std::vector<std::pair<double, const DMps*>>& terms,
                 int cap, Arena& out, hipStream_t s, double tol = -1.0);
  Arena& scratch() { return tmp_; }

 private:
  void absorb_left(const VSite& v, const double* R, int p, double* M,
                   hipStream_t s);
  DMps initial_state(int rank, const double* ax, const double* bv, hipStream_t s);
  void set_states_host(const std::vector<int>& bonds,
                       const std::vector<std::vector<double>>& packed, hipStream_t s);
  DMps stage_packed(const std::vector<int>& bonds, const std::vector<const double*>& packed,
                    hipStream_t s);
  void compress_right_half(DMps& res, int centre, const double* sc, int cap,
                           double tol, Arena& out, hipStream_t s,
                           std::vector<double>* disc);
  // centre site of the problem's compression scheme for an n-site chain
  int centre_for(int n) const {
    return (p_.compression == 1 && n == p_.n()) ? p_.Lx : 0;
  }
  void absorb_right(const VSite& v, const double* L, int q, double* N,
                    hipStream_t s);
  // n(x) = dv <1, g>_v, or dv <w, g>_v with the full-chain weight MPS
  // 1(x) w(v) (chain order) when wt is given
  DMps density(const DMps& g, Arena& ar, hipStream_t s, const DMps* wt = nullptr);
  // a function of x on the grid (device, natural bit order) as an x-MPS:
  // iterated SVD from the right with relative cut `cut`
  DMps vector_mps(const double* u, int L, double cut, Arena& ar, hipStream_t s);
  // the collision terms that depend on the moments of g (coll_model 0):
  // -nu (diag(v0) (x) Dv) g and nu (diag(vth^2) (x) Dv Dv) g, compressed
  void moment_collision_terms(const DMps& g, Arena& out, hipStream_t s,
                              DMps& Tu, DMps& Tt);
  DMps field(const DMps& g, Arena& ar, hipStream_t s);
  // diag(scale * X) (x) vop as a full-chain MPO, X an x-MPS (natural bit
  // order), vop a v-site MPO in chain order (the field term: X = E,
  // scale = -q/m, vop = Dv)
  DMpo t2_mpo(const DMps& X, Arena& ar, hipStream_t s, double scale, const DMpo& vop);
  DMps rhs(const DMps& g, Arena& out, hipStream_t s, const DMps* Eext = nullptr);
  DMps direct_sum(const std::vector<std::pair<double, const DMps*>>& t, Arena& ar,
                  hipStream_t s);
  void check_finite(const DMps& fn, hipStream_t s);
  void install(const DMps& fn, hipStream_t s);
  // the four RK4 stages of one step; the new state is left in staged_
  void step_stages(double h, hipStream_t s);
  void step_eager(double h, hipStream_t s);
  void step_capture(double h, hipStream_t s);
  void step_replay(hipStream_t s);
  bool graph_eligible() const;
  static bool same_cores(const std::vector<Core>& a, const std::vector<Core>& b);
  DMps copy_mps(const DMps& a, Arena& ar, hipStream_t s);
  DMps reverse_mps(const DMps& a, Arena& ar, hipStream_t s);
  void commit(const DMps& fn, hipStream_t s);
  double full_contract(const DMps& g, const DMps& f, hipStream_t s);
  void dense_of(const DMps& a, double* out, hipStream_t s);
  int cap_for(int point) const;
  // Compression workspace of the calling thread: work_ on the thread that
  // drives the engine, work2_ on the side thread of rhs().
  Arena& work();
  // the SVD outcome record of the lane whose stream is s
  SvdOutcomes* outcomes(hipStream_t s) { return s == side_ ? &out_side_ : &out_main_; }
  // launches over every instance, or over instance i alone
  Lanes all_lanes() const { return Lanes{nin_, 0, (long)chunk_, p_.tall_apply}; }
  Lanes one_lane(int i) const {
    return Lanes{1, (long)i * (long)chunk_, (long)chunk_, p_.tall_apply};
  }
  void check_instance(int i) const;
  // arithmetic of the MPO x MPS contractions: 0 FP64, 1 FP32, 2 BF16 on the
  // matrix cores (precision mode); factorisations, Poisson field and moments
  // stay FP64
  int contract_prec() const { return p_.precision; }

  Problem p_;                      // instance 0's problem
  std::vector<Problem> ps_;        // every instance's problem
  int nin_;                        // lock-step instances
  // chunk size of the arenas, scaled to the problem (see memory_model);
  // also the distance between two instances' copies of every buffer
  size_t chunk_;
  Arena ops_{chunk_, nin_};        // operators (persistent)
  Arena state_{chunk_, nin_};      // committed state
  Arena step_{chunk_, nin_};       // per-step intermediates
  Arena tmp_{chunk_, nin_};        // per-RHS intermediates
  Arena work_{chunk_, nin_};       // per-compression workspace
  Arena tmp2_{chunk_, nin_};       // per-RHS intermediates of the side lane
  Arena work2_{chunk_, nin_};      // compression workspace of the side lane
  int device_ = 0;                 // the device the instance lives on
  hipStream_t own_ = nullptr;      // this instance's stream (batched mode)
  hipStream_t side_ = nullptr;     // T1 runs here, beside T2
  hipEvent_t ev_fork_ = nullptr, ev_join_ = nullptr;
  hipEvent_t ev_in_ = nullptr, ev_out_ = nullptr;  // caller stream <-> own_
  // captured step graph and what it was captured for
  bool graph_on_ = false;
  hipGraphExec_t gexec_ = nullptr;
  std::vector<Core> graph_key_, warm_key_;  // input state layouts
  DMps graph_out_;                           // the graph's new state
  // SVD outcomes of the two lanes and their records kept for graph replays
  SvdOutcomes out_main_, out_side_;
  SvdOutcomes::Record rec_own_, rec_side_;
  bool capturing_ = false;         // a step graph is being recorded
  long graph_captures_ = 0, graph_replays_ = 0;
  DMpo t1_, gneg_, dv_;            // T1 chain, -G (x sites), Dv (v sites)
  DMpo coll_;                      // collision operator chain (nu > 0)
  DMpo dv2_;                       // Dv Dv on the v sites (moment collisions)
  DMps vpoly_, v2poly_;            // moment weights (full chain)
  DMps f_;
  DMps staged_;  // the new state of the step in flight (step_ arena)
  std::vector<double> disc_;
  double t_ = 0.0;
  long steps_ = 0;
  int* dflag_ = nullptr;
  PinnedBuf flags_host_;  // the finiteness flags of every instance
  // a kIdent x kIdent identity (device), for the exact gauges of the sweep
  static constexpr int kIdent = 256;
  double* ident_ = nullptr;
};

// Host construction of the operators (exact, FP64).  W[bl][o][i][br].
namespace ops {
using HostMpo = std::vector<std::vector<double>>;
HostMpo d1_periodic(int L, double h, std::vector<int>& bonds);
HostMpo d1_zero_gradient(int L, double h, std::vector<int>& bonds);
HostMpo poisson_g(int L, double dx, double scale, std::vector<int>& bonds);
// periodic second-order one-sided d/dx: forward (-3 f_i + 4 f_{i+1} -
// f_{i+2}) / 2h or backward (3 f_i - 4 f_{i-1} + f_{i-2}) / 2h, bond 3
HostMpo d1_one_sided(int L, double h, bool forward, std::vector<int>& bonds);
// diag(max(v_j, 0)) (positive) or diag(min(v_j, 0)), v_j = v0 + j dv
HostMpo velocity_part_diag(int L, double v0, double dv, bool positive,
                           std::vector<int>& bonds);
// direct sum of two MPOs of the same length (their operators add)
HostMpo mpo_add(const HostMpo& A, const std::vector<int>& ba, const HostMpo& B,
                const std::vector<int>& bb, std::vector<int>& bonds);
// diag of c0 + c1 J + c2 J^2 with J the integer index (MSB first); J -> v
HostMpo poly_diag(int L, double c0, double c1, double c2, std::vector<int>& bonds);
// the matching MPS (values instead of a diagonal operator)
std::vector<std::vector<double>> poly_mps(int L, double c0, double c1, double c2,
                                          std::vector<int>& bonds);
HostMpo chain(const HostMpo& Wx, const std::vector<int>& bx, const HostMpo& Wv,
              const std::vector<int>& bv, int order, std::vector<int>& bonds);
// operator product A B, bonds multiplied (A-major)
HostMpo mpo_product(const HostMpo& A, const std::vector<int>& ba, const HostMpo& B,
                    const std::vector<int>& bb, std::vector<int>& bonds);
// the same chain read from its last site: cores (l, P, r) -> (r, P, l)
HostMpo reverse(const HostMpo& W, const std::vector<int>& bonds, int P,
                std::vector<int>& out_bonds);
}  // namespace ops

}  // namespace mpsv
