// C-ABI of the MPS Vlasov-Poisson library (include/mps_vlasov.h and
// include/mps_blocks.h).  Converts engine exceptions into status codes and a
// thread-local message; no exception crosses the boundary.
#include <algorithm>
#include <atomic>
#include <exception>
#include <thread>
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>

#include "../../include/mps_blocks.h"
#include "../../include/mps_vlasov.h"
#include "engine.hpp"
#include "gemm.hpp"
#include "linalg.hpp"
#include "noalloc.hpp"
#include "prof.hpp"
#include "tune.hpp"

struct mps_state {
  std::shared_ptr<mpsv::Engine> eng;
  int device = 0;
  bool in_plasma = false;  // owned by an mps_plasma (mps_free refuses it)
  bool in_batch = false;   // a view of one instance of an mps_batch
  int inst = 0;            // its instance index
};

struct mps_batch {
  std::shared_ptr<mpsv::Engine> eng;
  std::vector<mps_state*> views;  // owned, one per instance
  int device = 0;
  ~mps_batch() {
    for (auto* h : views) delete h;
  }
};

struct mps_plasma {
  std::vector<mps_state*> species;  // owned
  std::vector<double> charge;
  int device = 0;
  ~mps_plasma() {
    for (auto* h : species) delete h;
  }
};

namespace {

thread_local std::string g_err;

mps_status to_status(int code) {
  switch (code) {
    case mpsv::kEinval: return MPS_EINVAL;
    case mpsv::kEnomem: return MPS_ENOMEM;
    case mpsv::kEnumeric: return MPS_ENUMERIC;
    default: return MPS_EDEVICE;
  }
}

template <class F>
mps_status guarded(F&& f) {
  try {
    g_err.clear();
    f();
    return MPS_OK;
  } catch (const mpsv::Error& e) {
    g_err = e.what();
    return to_status(e.code);
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return MPS_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return MPS_EDEVICE;
  } catch (...) {
    g_err = "unknown failure";
    return MPS_EDEVICE;
  }
}

mpsv::Problem convert(const mps_problem* p) {
  MPSV_CHECK(p != nullptr, mpsv::kEinval, "problem is NULL");
  mpsv::Problem q;
  q.Lx = p->Lx;
  q.Lv = p->Lv;
  q.order = p->order;
  q.x_min = p->x_min;
  q.x_max = p->x_max;
  q.v_min = p->v_min;
  q.v_max = p->v_max;
  q.qm = p->qm;
  q.dt = p->dt;
  q.chi_max = p->chi_max;
  q.level = p->level;
  q.df_max = p->df_max;
  q.tol = p->tol;
  q.precision = p->precision;
  q.x_scheme = p->x_scheme;
  q.cfl = p->cfl;
  q.compression = p->compression;
  q.nu = p->nu;
  q.nu_v0 = p->nu_v0;
  q.nu_vth = p->nu_vth;
  q.coll_model = p->coll_model;
  q.tall_apply = p->tall_apply;
  MPSV_CHECK(std::isfinite(q.x_min) && std::isfinite(q.x_max) &&
                 std::isfinite(q.v_min) && std::isfinite(q.v_max),
             mpsv::kEinval, "grid bounds must be finite");
  return q;
}

void check_handle(const mps_state* h) {
  MPSV_CHECK(h != nullptr && h->eng, mpsv::kEinval, "state handle is NULL");
  int dev = -1;
  MPSV_HIP(hipGetDevice(&dev));
  MPSV_CHECK(dev == h->device, mpsv::kEinval,
             "state was created on another device than the current one");
}

// A small engine whose arenas serve the stand-alone building blocks.
std::mutex g_blocks_mu;
std::unique_ptr<mpsv::Engine> g_blocks;
mpsv::Engine& blocks() {
  if (!g_blocks) {
    mpsv::Problem p;
    p.Lx = p.Lv = 2;
    p.x_min = 0;
    p.x_max = 1;
    p.v_min = -1;
    p.v_max = 1;
    g_blocks.reset(new mpsv::Engine(p));
  }
  return *g_blocks;
}

mpsv::DMps unpack(int n, const int32_t* bonds, const double* cores) {
  MPSV_CHECK(bonds != nullptr && cores != nullptr, mpsv::kEinval,
             "bonds / cores must not be NULL");
  MPSV_CHECK(bonds[0] == 1 && bonds[n] == 1, mpsv::kEinval,
             "end bonds must be 1");
  mpsv::DMps a(n);
  long off = 0;
  for (int j = 0; j < n; ++j) {
    MPSV_CHECK(bonds[j + 1] >= 1, mpsv::kEinval, "bond dimension must be >= 1");
    a[j] = mpsv::Core{const_cast<double*>(cores) + off, bonds[j], bonds[j + 1]};
    off += a[j].size();
  }
  return a;
}

void pack(const mpsv::DMps& a, int32_t* bonds, double* out, int64_t capacity,
          hipStream_t s) {
  long tot = 0;
  for (auto& c : a) tot += c.size();
  MPSV_CHECK(tot <= capacity, mpsv::kEinval,
             "output capacity too small: need " + std::to_string(tot));
  long off = 0;
  bonds[0] = 1;
  for (size_t j = 0; j < a.size(); ++j) {
    bonds[j + 1] = a[j].r;
    MPSV_HIP(hipMemcpyAsync(out + off, a[j].p, a[j].size() * sizeof(double),
                            hipMemcpyDeviceToDevice, s));
    off += a[j].size();
  }
  MPSV_HIP(hipStreamSynchronize(s));
}

}  // namespace

extern "C" {

const char* mps_last_error(void) { return g_err.c_str(); }

mps_status mps_init(const mps_problem* p, int32_t rank, const double* ax,
                    const double* bv, hipStream_t stream, mps_state** out) {
  return guarded([&] {
    MPSV_CHECK(out != nullptr, mpsv::kEinval, "out is NULL");
    *out = nullptr;
    MPSV_CHECK(ax != nullptr && bv != nullptr, mpsv::kEinval,
               "profiles must not be NULL");
    mpsv::Problem q = convert(p);
    std::unique_ptr<mps_state> h(new mps_state);
    MPSV_HIP(hipGetDevice(&h->device));
    h->eng.reset(new mpsv::Engine(q));
    h->eng->init_from_profiles(rank, ax, bv, stream);
    *out = h.release();
  });
}

mps_status mps_step(mps_state* h, int32_t nsteps, hipStream_t stream) {
  return guarded([&] {
    check_handle(h);
    MPSV_CHECK(nsteps >= 0, mpsv::kEinval, "nsteps must be >= 0");
    MPSV_CHECK(!h->in_plasma, mpsv::kEinval,
               "a species of a plasma is stepped by mps_plasma_step");
    MPSV_CHECK(!h->in_batch, mpsv::kEinval,
               "an instance of a batch is stepped by mps_batch_step");
    for (int i = 0; i < nsteps; ++i) h->eng->step(stream);
  });
}

mps_status mps_moments(mps_state* h, double* n_out, double* E_out,
                       double* scalars, hipStream_t stream) {
  return guarded([&] {
    check_handle(h);
    h->eng->moments(n_out, E_out, scalars, stream, h->inst);
  });
}

mps_status mps_to_dense(mps_state* h, double* f_out, hipStream_t stream) {
  return guarded([&] {
    check_handle(h);
    MPSV_CHECK(f_out != nullptr, mpsv::kEinval, "f_out is NULL");
    h->eng->to_dense(f_out, stream, h->inst);
    MPSV_HIP(hipStreamSynchronize(stream));
  });
}

mps_status mps_free(mps_state* h) {
  return guarded([&] {
    if (!h) return;
    MPSV_CHECK(!h->in_plasma, mpsv::kEinval,
               "a species of a plasma is released by mps_plasma_free");
    MPSV_CHECK(!h->in_batch, mpsv::kEinval,
               "an instance of a batch is released by mps_batch_free");
    (void)hipDeviceSynchronize();
    delete h;
  });
}

mps_status mps_info(const mps_state* h, int32_t* n_sites, int32_t* bond_dims,
                    double* discarded, double* t, int64_t* steps) {
  return guarded([&] {
    check_handle(h);
    const mpsv::Engine& e = *h->eng;
    if (n_sites) *n_sites = e.n();
    if (bond_dims) {
      auto b = e.bonds();
      for (size_t j = 0; j < b.size(); ++j) bond_dims[j] = b[j];
    }
    if (discarded) {
      const auto d = e.last_discarded(h->inst);
      for (int j = 0; j < e.n() - 1; ++j)
        discarded[j] = j < (int)d.size() ? d[j] : 0.0;
    }
    if (t) *t = e.time();
    if (steps) *steps = e.steps_done();
  });
}

mps_status mps_get_cores(const mps_state* h, int32_t* bond_dims,
                         int64_t* count, double* cores, hipStream_t stream) {
  return guarded([&] {
    check_handle(h);
    std::vector<int> b;
    h->eng->get_state(b, cores, stream, h->inst);
    long tot = 0;
    for (size_t j = 0; j + 1 < b.size(); ++j) tot += (long)b[j] * 2 * b[j + 1];
    if (bond_dims)
      for (size_t j = 0; j < b.size(); ++j) bond_dims[j] = b[j];
    if (count) *count = tot;
    MPSV_HIP(hipStreamSynchronize(stream));
  });
}

mps_status mps_set_cores(mps_state* h, const int32_t* bond_dims,
                         const double* cores, hipStream_t stream) {
  return guarded([&] {
    check_handle(h);
    MPSV_CHECK(bond_dims && cores, mpsv::kEinval, "NULL argument");
    MPSV_CHECK(!h->in_batch, mpsv::kEinval,
               "the instances of a batch take their cores by mps_batch_set_cores");
    std::vector<int> b(bond_dims, bond_dims + h->eng->n() + 1);
    h->eng->set_state(b, cores, stream);
  });
}

mps_status mps_add_scaled(mps_state* h, double alpha, const int32_t* bond_dims,
                          const double* cores, hipStream_t stream) {
  return guarded([&] {
    check_handle(h);
    MPSV_CHECK(bond_dims && cores, mpsv::kEinval, "NULL argument");
    MPSV_CHECK(std::isfinite(alpha), mpsv::kEinval, "alpha must be finite");
    MPSV_CHECK(!h->in_batch, mpsv::kEinval,
               "the instances of a batch are perturbed by mps_batch_add_scaled");
    std::vector<int> b(bond_dims, bond_dims + h->eng->n() + 1);
    h->eng->add_scaled(alpha, b, cores, stream);
  });
}

mps_status mps_workspace_bound(const mps_problem* p, size_t* bytes) {
  return guarded([&] {
    MPSV_CHECK(bytes != nullptr, mpsv::kEinval, "bytes is NULL");
    mpsv::Problem q = convert(p);
    mpsv::validate_problem(q);
    *bytes = mpsv::memory_model(q).bound;
  });
}

mps_status mps_entanglement(mps_state* h, double* ee, hipStream_t stream) {
  return guarded([&] {
    check_handle(h);
    MPSV_CHECK(ee != nullptr, mpsv::kEinval, "ee is NULL");
    auto v = h->eng->entanglement(stream, h->inst);
    for (size_t j = 0; j < v.size(); ++j) ee[j] = v[j];
  });
}

mps_status mps_device_bytes(const mps_state* h, size_t* bytes) {
  return guarded([&] {
    check_handle(h);
    MPSV_CHECK(bytes != nullptr, mpsv::kEinval, "bytes is NULL");
    *bytes = h->eng->device_bytes();
  });
}

mps_status mpsb_arena_bytes(const mps_state* h, size_t* reserved, size_t* peak) {
  return guarded([&] {
    check_handle(h);
    MPSV_CHECK(reserved != nullptr && peak != nullptr, mpsv::kEinval, "NULL argument");
    h->eng->arena_bytes(reserved, peak);
  });
}

mps_status mps_step_batched(mps_state* const* hs, int32_t count, int32_t nsteps,
                            hipStream_t stream) {
  return guarded([&] {
    MPSV_CHECK(hs != nullptr && count >= 0, mpsv::kEinval, "bad batch");
    MPSV_CHECK(nsteps >= 0, mpsv::kEinval, "nsteps must be >= 0");
    for (int i = 0; i < count; ++i) {
      check_handle(hs[i]);
      MPSV_CHECK(!hs[i]->in_plasma, mpsv::kEinval,
                 "a species of a plasma is stepped by mps_plasma_step");
      MPSV_CHECK(!hs[i]->in_batch, mpsv::kEinval,
                 "an instance of a batch is stepped by mps_batch_step");
    }
    {
      std::vector<const mps_state*> v(hs, hs + count);
      std::sort(v.begin(), v.end());
      MPSV_CHECK(std::adjacent_find(v.begin(), v.end()) == v.end(),
                 mpsv::kEinval, "a batch must not list an instance twice");
    }
    if (count == 0 || nsteps == 0) return;
    int dev = 0;
    MPSV_HIP(hipGetDevice(&dev));
    // Every instance runs on its own stream, driven by its own host thread
    // (at most 16 at a time); the caller's stream is ordered before and
    // after all of them.
    hipEvent_t start;
    MPSV_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
    MPSV_HIP(hipEventRecord(start, stream));
    for (int i = 0; i < count; ++i)
      MPSV_HIP(hipStreamWaitEvent(hs[i]->eng->own_stream(), start, 0));
    std::vector<std::exception_ptr> errs(count);
    std::atomic<int> next{0};
    auto worker = [&] {
      (void)hipSetDevice(dev);
      for (;;) {
        const int i = next++;
        if (i >= count) break;
        try {
          for (int k = 0; k < nsteps; ++k)
            hs[i]->eng->step(hs[i]->eng->own_stream());
        } catch (...) {
          errs[i] = std::current_exception();
        }
      }
    };
    const int nt = std::min(count, 16);
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t) pool.emplace_back(worker);
    for (auto& t : pool) t.join();
    for (int i = 0; i < count; ++i) {
      hipEvent_t done;
      MPSV_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
      MPSV_HIP(hipEventRecord(done, hs[i]->eng->own_stream()));
      MPSV_HIP(hipStreamWaitEvent(stream, done, 0));
      MPSV_HIP(hipEventDestroy(done));
    }
    MPSV_HIP(hipEventDestroy(start));
    for (int i = 0; i < count; ++i)
      if (errs[i]) {
        try {
          std::rethrow_exception(errs[i]);
        } catch (const mpsv::Error& e) {
          throw mpsv::Error(e.code, "instance " + std::to_string(i) + ": " + e.what());
        }
      }
  });
}

// ------------------------------------------------------------- blocks

mps_status mpsb_gemm(int32_t M, int32_t N, int32_t K, double alpha,
                     const double* A, int64_t lda, const double* B,
                     int64_t ldb, double beta, double* C, int64_t ldc,
                     hipStream_t stream) {
  return mpsb_gemm_prec(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                        MPS_PREC_FP64, stream);
}

mps_status mpsb_gemm_prec(int32_t M, int32_t N, int32_t K, double alpha,
                          const double* A, int64_t lda, const double* B,
                          int64_t ldb, double beta, double* C, int64_t ldc,
                          int32_t precision, hipStream_t stream) {
  return guarded([&] {
    MPSV_CHECK(M >= 0 && N >= 0 && K >= 0, mpsv::kEinval, "negative size");
    MPSV_CHECK(lda >= K && ldb >= N && ldc >= N, mpsv::kEinval,
               "leading dimension too small");
    MPSV_CHECK(precision == MPS_PREC_FP64 || precision == MPS_PREC_FP32_CONTRACT ||
                   precision == MPS_PREC_BF16_CONTRACT,
               mpsv::kEinval, "unknown precision");
    std::lock_guard<std::mutex> lk(g_blocks_mu);
    mpsv::gemm(stream, M, N, K, alpha, mpsv::CMatView{A, lda, 1, 0},
               mpsv::CMatView{B, ldb, 1, 0}, beta, mpsv::MatView{C, ldc, 1, 0},
               1, (int)precision, &blocks().scratch());
    MPSV_HIP(hipStreamSynchronize(stream));
  });
}

mps_status mpsb_gemm_strided(int32_t M, int32_t N, int32_t K, double alpha,
                             const double* A, int64_t ars, int64_t acs, int64_t abs_,
                             const double* B, int64_t brs, int64_t bcs, int64_t bbs,
                             double beta, double* C, int64_t crs, int64_t ccs,
                             int64_t cbs, int32_t batch, int32_t precision,
                             hipStream_t stream) {
  return guarded([&] {
    MPSV_CHECK(M >= 0 && N >= 0 && K >= 0 && batch >= 0, mpsv::kEinval, "negative size");
    MPSV_CHECK(A && B && C, mpsv::kEinval, "NULL operand");
    MPSV_CHECK(precision == MPS_PREC_FP64 || precision == MPS_PREC_FP32_CONTRACT ||
                   precision == MPS_PREC_BF16_CONTRACT,
               mpsv::kEinval, "unknown precision");
    std::lock_guard<std::mutex> lk(g_blocks_mu);
    mpsv::gemm(stream, M, N, K, alpha, mpsv::CMatView{A, ars, acs, abs_},
               mpsv::CMatView{B, brs, bcs, bbs}, beta, mpsv::MatView{C, crs, ccs, cbs},
               batch, (int)precision, &blocks().scratch());
    MPSV_HIP(hipStreamSynchronize(stream));
  });
}

mps_status mpsb_qr(int32_t m, int32_t n, double* A, double* Q,
                   hipStream_t stream) {
  return mpsb_qr_tall(m, n, A, Q, MPS_TALL_APPLY_REFLECTORS, stream);
}

mps_status mpsb_qr_tall(int32_t m, int32_t n, double* A, double* Q,
                        int32_t tall_apply, hipStream_t stream) {
  return guarded([&] {
    MPSV_CHECK(m >= 1 && n >= 1 && A, mpsv::kEinval, "bad QR arguments");
    MPSV_CHECK(tall_apply == MPS_TALL_APPLY_REFLECTORS || tall_apply == MPS_TALL_APPLY_WY,
               mpsv::kEinval, "tall_apply must be 0 or 1");
    mpsv::Lanes l;
    l.tall_apply = tall_apply;
    mpsv::LanesScope ls(l);
    std::lock_guard<std::mutex> lk(g_blocks_mu);
    mpsv::Arena& ws = blocks().scratch();
    mpsv::ArenaScope sc(ws);
    mpsv::QrFactor f;
    mpsv::qr_factor(stream, ws, A, m, n, n, f);
    if (Q) {
      const int k = std::min(m, n);
      // Q = H_0 ... H_{k-1} [I_k; 0], the identity read through a view
      // (rows past k enter as zeros), as the compression sweeps apply Q
      double* E = ws.alloc((size_t)k * k);
      std::vector<double> h((size_t)k * k, 0.0);
      for (int i = 0; i < k; ++i) h[(size_t)i * k + i] = 1.0;
      MPSV_HIP(hipMemcpy(E, h.data(), h.size() * sizeof(double),
                         hipMemcpyHostToDevice));
      mpsv::qr_apply_q_view(stream, ws, f, mpsv::CMatView{E, k, 1, 0}, k,
                            mpsv::MatView{Q, k, 1, 0}, k);
    }
    MPSV_HIP(hipStreamSynchronize(stream));
  });
}

mps_status mpsb_svd_truncate(int32_t m, int32_t c, double* X, int32_t cap,
                             double tol, double* Vt, double* US, double* sig,
                             int32_t* D, double* discarded,
                             hipStream_t stream) {
  return guarded([&] {
    MPSV_CHECK(m >= 1 && c >= 1 && X && Vt && US && D, mpsv::kEinval,
               "bad SVD arguments");
    MPSV_CHECK(tol >= 0, mpsv::kEinval, "tol must be >= 0");
    std::lock_guard<std::mutex> lk(g_blocks_mu);
    mpsv::Arena& ws = blocks().scratch();
    mpsv::ArenaScope sc(ws);
    double dsc = 0;
    *D = mpsv::svd_truncate(stream, ws, X, m, c, c, cap > 0 ? cap : INT_MAX,
                            tol, Vt, US, sig, &dsc);
    if (discarded) *discarded = dsc;
    MPSV_HIP(hipStreamSynchronize(stream));
  });
}

mps_status mpsb_svd_truncate_noalloc(int32_t m, int32_t c, double* X, int32_t cap,
                                     double tol, double* Vt, double* US, double* sig,
                                     int32_t* D, double* discarded,
                                     hipStream_t stream) {
  return guarded([&] {
    MPSV_CHECK(m >= 1 && c >= 1 && X && Vt && US && D, mpsv::kEinval,
               "bad SVD arguments");
    MPSV_CHECK(tol >= 0, mpsv::kEinval, "tol must be >= 0");
    MPSV_CHECK(m <= 2048 && c <= 2048 && std::min(m, c) <= 256, mpsv::kEinval,
               "mpsb_svd_truncate_noalloc takes m, c <= 2048 and min(m, c) <= 256 "
               "(its fixed device scratch is " +
                   std::to_string(mpsv::kNoAllocScratchBytes >> 20) + " MiB)");
    // one call at a time per process: every call on a GPU shares its
    // scratch, and a call ends only after its stream has completed
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    mpsv::Arena ws(mpsv::noalloc_scratch(), mpsv::kNoAllocScratchBytes);
    double dsc = 0;
    *D = mpsv::svd_truncate(stream, ws, X, m, c, c, cap > 0 ? cap : INT_MAX,
                            tol, Vt, US, sig, &dsc);
    if (discarded) *discarded = dsc;
    MPSV_HIP(hipStreamSynchronize(stream));
  });
}

mps_status mpsb_compress(int32_t n, const int32_t* mpo_bonds,
                         const double* mpo, const int32_t* bonds_in,
                         const double* cores_in, int32_t cap, double tol,
                         int32_t* bonds_out, double* cores_out,
                         int64_t capacity, double* discarded,
                         hipStream_t stream) {
  return guarded([&] {
    MPSV_CHECK(n >= 2 && n <= 28, mpsv::kEinval, "n must lie in [2, 28]");
    MPSV_CHECK(tol >= 0, mpsv::kEinval, "tol must be >= 0");
    MPSV_CHECK(bonds_out && cores_out, mpsv::kEinval, "NULL output");
    std::lock_guard<std::mutex> lk(g_blocks_mu);
    mpsv::Engine& e = blocks();
    mpsv::Arena out;
    mpsv::DMps a = unpack(n, bonds_in, cores_in);
    std::vector<double> disc;
    mpsv::DMps r;
    if (mpo) {
      MPSV_CHECK(mpo_bonds && mpo_bonds[0] == 1 && mpo_bonds[n] == 1,
                 mpsv::kEinval, "bad MPO bonds");
      std::vector<std::vector<double>> W(n);
      std::vector<int> wb(mpo_bonds, mpo_bonds + n + 1);
      long off = 0;
      for (int j = 0; j < n; ++j) {
        W[j].resize((size_t)wb[j] * 4 * wb[j + 1]);
        MPSV_HIP(hipMemcpy(W[j].data(), mpo + off, W[j].size() * sizeof(double),
                           hipMemcpyDeviceToHost));
        off += W[j].size();
      }
      mpsv::DMpo dW = e.upload_mpo(W, wb, out, stream);
      r = e.apply_compress(dW, a, cap > 0 ? cap : INT_MAX, tol, out, stream,
                           &disc);
    } else {
      r = e.compress_mps(a, cap > 0 ? cap : INT_MAX, tol, out, stream, &disc);
    }
    pack(r, bonds_out, cores_out, capacity, stream);
    if (discarded)
      for (int j = 0; j < n - 1; ++j) discarded[j] = disc[j];
  });
}

mps_status mpsb_step_graph(mps_state* h, int32_t enable, int64_t* captures,
                           int64_t* replays) {
  return guarded([&] {
    check_handle(h);
    MPSV_CHECK(!h->in_plasma && !h->in_batch, mpsv::kEinval,
               "step graphs belong to stand-alone states");
    if (enable >= 0) h->eng->set_step_graph(enable != 0);
    if (captures) *captures = h->eng->graph_captures();
    if (replays) *replays = h->eng->graph_replays();
  });
}

mps_status mpsb_compress_centre(int32_t n, int32_t centre,
                                const int32_t* bonds_in, const double* cores_in,
                                int32_t cap, double tol, int32_t* bonds_out,
                                double* cores_out, int64_t capacity,
                                double* discarded, hipStream_t stream) {
  return guarded([&] {
    MPSV_CHECK(n >= 2 && n <= 28, mpsv::kEinval, "n must lie in [2, 28]");
    MPSV_CHECK(centre >= 1 && centre <= n - 1, mpsv::kEinval,
               "centre must lie in [1, n-1]");
    MPSV_CHECK(tol >= 0, mpsv::kEinval, "tol must be >= 0");
    MPSV_CHECK(bonds_out && cores_out, mpsv::kEinval, "NULL output");
    std::lock_guard<std::mutex> lk(g_blocks_mu);
    mpsv::Engine& e = blocks();
    mpsv::Arena out;
    mpsv::DMps a = unpack(n, bonds_in, cores_in);
    std::vector<double> disc;
    mpsv::DMps r = e.compress_mps(a, cap > 0 ? cap : INT_MAX, tol, out, stream,
                                  &disc, centre);
    pack(r, bonds_out, cores_out, capacity, stream);
    if (discarded)
      for (int j = 0; j < n - 1; ++j) discarded[j] = disc[j];
  });
}

mps_status mpsb_add_compress(int32_t n, int32_t nterms, const double* coef,
                             const int32_t* bonds, const double* const* cores,
                             int32_t cap, double tol, int32_t* bonds_out,
                             double* cores_out, int64_t capacity,
                             hipStream_t stream) {
  return guarded([&] {
    MPSV_CHECK(n >= 2 && nterms >= 1 && coef && bonds && cores, mpsv::kEinval,
               "bad arguments");
    std::lock_guard<std::mutex> lk(g_blocks_mu);
    mpsv::Engine& e = blocks();
    mpsv::Arena out;
    std::vector<mpsv::DMps> terms;
    for (int t = 0; t < nterms; ++t)
      terms.push_back(unpack(n, bonds + (long)t * (n + 1), cores[t]));
    std::vector<std::pair<double, const mpsv::DMps*>> tl;
    for (int t = 0; t < nterms; ++t) tl.push_back({coef[t], &terms[t]});
    mpsv::DMps r = e.add_terms(tl, cap > 0 ? cap : INT_MAX, out, stream, tol);
    pack(r, bonds_out, cores_out, capacity, stream);
  });
}

mps_status mpsb_density_field(mps_state* h, double* n_out, double* E_out,
                              hipStream_t stream) {
  return guarded([&] {
    check_handle(h);
    h->eng->density_field(n_out, E_out, stream, h->inst);
  });
}

mps_status mpsb_operator(int32_t which, int32_t L, double h0, double h,
                         int32_t* bonds, double* W, int64_t* count) {
  return guarded([&] {
    MPSV_CHECK(L >= 2 && L <= 14, mpsv::kEinval, "L must lie in [2, 14]");
    std::vector<int> b;
    mpsv::ops::HostMpo M;
    switch (which) {
      case 0: M = mpsv::ops::d1_periodic(L, h, b); break;
      case 1: M = mpsv::ops::d1_zero_gradient(L, h, b); break;
      case 2: M = mpsv::ops::poisson_g(L, h, 1.0, b); break;
      case 3: M = mpsv::ops::poly_diag(L, h0, h, 0.0, b); break;
      case 4: M = mpsv::ops::d1_one_sided(L, h, false, b); break;
      case 5: M = mpsv::ops::d1_one_sided(L, h, true, b); break;
      case 6: M = mpsv::ops::velocity_part_diag(L, h0, h, true, b); break;
      case 7: M = mpsv::ops::velocity_part_diag(L, h0, h, false, b); break;
      default: throw mpsv::Error(mpsv::kEinval, "unknown operator");
    }
    long tot = 0;
    for (auto& x : M) tot += (long)x.size();
    if (count) *count = tot;
    if (bonds)
      for (size_t j = 0; j < b.size(); ++j) bonds[j] = b[j];
    if (W) {
      long off = 0;
      for (auto& x : M) {
        std::memcpy(W + off, x.data(), x.size() * sizeof(double));
        off += (long)x.size();
      }
    }
  });
}

mps_status mpsb_stats(int64_t* qr_calls, int64_t* svd_calls,
                      int64_t* jacobi_sweeps) {
  return guarded([&] {
    auto& s = mpsv::linalg_stats();
    if (qr_calls) *qr_calls = s.qr_calls;
    if (svd_calls) *svd_calls = s.svd_calls;
    if (jacobi_sweeps) *jacobi_sweeps = s.jacobi_sweeps;
  });
}

mps_status mpsb_set_jacobi_max_sweeps(int32_t n) {
  return guarded([&] {
    MPSV_CHECK(n >= 1, mpsv::kEinval, "sweep cap must be >= 1");
    mpsv::set_jacobi_max_sweeps(n);
  });
}

mps_status mpsb_tune_clear(void) {
  return guarded([&] { mpsv::tune_clear(); });
}

static mpsv::TuneKey tune_key(const int32_t* key6) {
  MPSV_CHECK(key6 != nullptr, mpsv::kEinval, "tuning key missing");
  mpsv::TuneKey k;
  for (int i = 0; i < mpsv::kTuneKeyInts; ++i) k.v[i] = key6[i];
  return k;
}

mps_status mpsb_tune_set(const int32_t* key6, int32_t value) {
  return guarded([&] { mpsv::tune_set(tune_key(key6), value); });
}

mps_status mpsb_tune_get(const int32_t* key6, int32_t* value, int32_t* found) {
  return guarded([&] {
    int32_t v = 0;
    const bool f = mpsv::tune_get(tune_key(key6), &v);
    if (found) *found = f ? 1 : 0;
    if (value && f) *value = v;
  });
}

mps_status mpsb_tune_size(int64_t* n) {
  return guarded([&] {
    MPSV_CHECK(n != nullptr, mpsv::kEinval, "null output");
    *n = mpsv::tune_size();
  });
}

mps_status mpsb_tune_load(const char* path) {
  return guarded([&] {
    MPSV_CHECK(path != nullptr, mpsv::kEinval, "null path");
    mpsv::tune_load(path);
  });
}

mps_status mpsb_tune_save(const char* path) {
  return guarded([&] {
    MPSV_CHECK(path != nullptr, mpsv::kEinval, "null path");
    mpsv::tune_save(path);
  });
}

mps_status mpsb_tune_record(int32_t on) {
  return guarded([&] { mpsv::tune_record(on != 0); });
}

mps_status mpsb_tune_records(int32_t* keys, int32_t* values, uint32_t* allowed,
                             int64_t* launches, double* ms, int64_t cap,
                             int64_t* n) {
  return guarded([&] {
    MPSV_CHECK(cap >= 0 && n != nullptr, mpsv::kEinval, "bad record buffer");
    const auto r = mpsv::tune_records();
    *n = (int64_t)r.size();
    for (int64_t i = 0; i < (int64_t)r.size() && i < cap; ++i) {
      if (keys)
        for (int j = 0; j < mpsv::kTuneKeyInts; ++j) keys[i * mpsv::kTuneKeyInts + j] = r[i].key.v[j];
      if (values) values[i] = r[i].value;
      if (allowed) allowed[i] = r[i].allowed;
      if (launches) launches[i] = r[i].launches;
      if (ms) ms[i] = r[i].ms;
    }
  });
}

mps_status mpsb_profile(int32_t enable) {
  return guarded([&] { mpsv::prof_enable(enable != 0); });
}

mps_status mpsb_profile_nested_flops(int32_t cls, double* flops) {
  return guarded([&] {
    MPSV_CHECK(cls >= 0 && cls < mpsv::kClsCount, mpsv::kEinval, "bad class");
    MPSV_CHECK(flops != nullptr, mpsv::kEinval, "null output");
    *flops = mpsv::prof_nested_flops(cls);
  });
}

mps_status mpsb_profile_read(int32_t cls, int64_t* launches, double* ms,
                             double* flops, double* bytes) {
  return guarded([&] {
    MPSV_CHECK(cls >= 0 && cls < mpsv::kClsCount, mpsv::kEinval, "bad class");
    long n = 0;
    mpsv::prof_read(cls, &n, ms, flops, bytes);
    if (launches) *launches = n;
  });
}

}  // extern "C"

// ------------------------------------------------------------- batches

mps_status mps_batch_init(int32_t count, const mps_problem* problems,
                          const int32_t* ranks, const double* const* ax,
                          const double* const* bv, hipStream_t stream,
                          mps_batch** out) {
  return guarded([&] {
    MPSV_CHECK(out != nullptr, mpsv::kEinval, "out is NULL");
    *out = nullptr;
    MPSV_CHECK(count >= 1 && count <= 1024, mpsv::kEinval, "count must lie in [1, 1024]");
    MPSV_CHECK(problems && ranks && ax && bv, mpsv::kEinval, "NULL argument");
    std::vector<mpsv::Problem> qs;
    std::vector<int> rk;
    std::vector<const double*> a, b;
    for (int i = 0; i < count; ++i) {
      qs.push_back(convert(&problems[i]));
      MPSV_CHECK(ax[i] && bv[i], mpsv::kEinval, "profiles must not be NULL");
      rk.push_back(ranks[i]);
      a.push_back(ax[i]);
      b.push_back(bv[i]);
    }
    std::unique_ptr<mps_batch> bt(new mps_batch);
    MPSV_HIP(hipGetDevice(&bt->device));
    bt->eng = std::make_shared<mpsv::Engine>(qs);
    bt->eng->init_batch(rk, a, b, stream);
    for (int i = 0; i < count; ++i) {
      std::unique_ptr<mps_state> h(new mps_state);
      h->eng = bt->eng;
      h->device = bt->device;
      h->in_batch = true;
      h->inst = i;
      bt->views.push_back(h.release());
    }
    *out = bt.release();
  });
}

namespace {
mpsv::Engine& batch_engine(mps_batch* b) {
  MPSV_CHECK(b != nullptr && b->eng, mpsv::kEinval, "batch handle is NULL");
  int dev = -1;
  MPSV_HIP(hipGetDevice(&dev));
  MPSV_CHECK(dev == b->device, mpsv::kEinval,
             "batch was created on another device than the current one");
  return *b->eng;
}
}  // namespace

mps_status mps_batch_set_cores(mps_batch* b, const int32_t* bond_dims,
                               const double* const* cores, hipStream_t stream) {
  return guarded([&] {
    mpsv::Engine& e = batch_engine(b);
    MPSV_CHECK(bond_dims && cores, mpsv::kEinval, "NULL argument");
    std::vector<int> bd(bond_dims, bond_dims + e.n() + 1);
    std::vector<const double*> c(cores, cores + e.instances());
    for (auto* p : c) MPSV_CHECK(p != nullptr, mpsv::kEinval, "cores must not be NULL");
    e.set_states(bd, c, stream);
  });
}

mps_status mps_batch_add_scaled(mps_batch* b, const double* alpha,
                                const int32_t* bond_dims,
                                const double* const* cores, hipStream_t stream) {
  return guarded([&] {
    mpsv::Engine& e = batch_engine(b);
    MPSV_CHECK(alpha && bond_dims && cores, mpsv::kEinval, "NULL argument");
    std::vector<int> bd(bond_dims, bond_dims + e.n() + 1);
    std::vector<const double*> c(cores, cores + e.instances());
    for (auto* p : c) MPSV_CHECK(p != nullptr, mpsv::kEinval, "cores must not be NULL");
    std::vector<double> al(alpha, alpha + e.instances());
    e.add_scaled_all(al, bd, c, stream);
  });
}

mps_status mps_batch_step(mps_batch* b, int32_t nsteps, hipStream_t stream) {
  return guarded([&] {
    mpsv::Engine& e = batch_engine(b);
    MPSV_CHECK(nsteps >= 0, mpsv::kEinval, "nsteps must be >= 0");
    for (int i = 0; i < nsteps; ++i) e.step(stream);
  });
}

mps_status mpsb_batch_step_graph(mps_batch* b, int32_t enable, int64_t* captures,
                                 int64_t* replays) {
  return guarded([&] {
    mpsv::Engine& e = batch_engine(b);
    if (enable >= 0) e.set_step_graph(enable != 0);
    if (captures) *captures = e.graph_captures();
    if (replays) *replays = e.graph_replays();
  });
}

mps_state* mps_batch_instance(mps_batch* b, int32_t i) {
  if (!b || i < 0 || i >= (int32_t)b->views.size()) return nullptr;
  return b->views[(size_t)i];
}

mps_status mps_batch_free(mps_batch* b) {
  return guarded([&] {
    if (!b) return;
    (void)hipDeviceSynchronize();
    delete b;
  });
}

// ------------------------------------------------------------ plasmas

mps_status mps_plasma_init(int32_t n_species, const mps_problem* species,
                           const double* charges, const int32_t* ranks,
                           const double* const* ax, const double* const* bv,
                           hipStream_t stream, mps_plasma** out) {
  return guarded([&] {
    MPSV_CHECK(out != nullptr, mpsv::kEinval, "out is NULL");
    *out = nullptr;
    MPSV_CHECK(n_species >= 1 && n_species <= 8, mpsv::kEinval,
               "n_species must lie in [1, 8]");
    MPSV_CHECK(species && charges && ranks && ax && bv, mpsv::kEinval,
               "NULL argument");
    std::unique_ptr<mps_plasma> pl(new mps_plasma);
    MPSV_HIP(hipGetDevice(&pl->device));
    std::vector<mpsv::Problem> qs;
    for (int i = 0; i < n_species; ++i) qs.push_back(convert(&species[i]));
    const mpsv::Problem& a = qs[0];
    for (int i = 0; i < n_species; ++i) {
      const mpsv::Problem& b = qs[i];
      MPSV_CHECK(b.Lx == a.Lx && b.x_min == a.x_min && b.x_max == a.x_max,
                 mpsv::kEinval, "species must share the x grid");
      MPSV_CHECK(b.dt == a.dt && b.cfl == 0.0, mpsv::kEinval,
                 "species must share a fixed dt (cfl = 0)");
      MPSV_CHECK(b.tall_apply == a.tall_apply, mpsv::kEinval,
                 "species must share the reflector application mode");
      MPSV_CHECK(std::isfinite(charges[i]), mpsv::kEinval, "charge must be finite");
      MPSV_CHECK(ax[i] && bv[i], mpsv::kEinval, "profiles must not be NULL");
    }
    for (int i = 0; i < n_species; ++i) {
      std::unique_ptr<mps_state> h(new mps_state);
      h->device = pl->device;
      h->in_plasma = true;
      h->eng.reset(new mpsv::Engine(qs[i]));
      h->eng->init_from_profiles(ranks[i], ax[i], bv[i], stream);
      pl->species.push_back(h.release());
      pl->charge.push_back(charges[i]);
    }
    *out = pl.release();
  });
}

namespace {
std::vector<mpsv::Engine*> engines_of(mps_plasma* pl) {
  MPSV_CHECK(pl != nullptr && !pl->species.empty(), mpsv::kEinval,
             "plasma handle is NULL");
  int dev = -1;
  MPSV_HIP(hipGetDevice(&dev));
  MPSV_CHECK(dev == pl->device, mpsv::kEinval,
             "plasma was created on another device than the current one");
  std::vector<mpsv::Engine*> es;
  for (auto* h : pl->species) es.push_back(h->eng.get());
  return es;
}
}  // namespace

mps_status mps_plasma_step(mps_plasma* pl, int32_t nsteps, hipStream_t stream) {
  return guarded([&] {
    auto es = engines_of(pl);
    MPSV_CHECK(nsteps >= 0, mpsv::kEinval, "nsteps must be >= 0");
    for (int i = 0; i < nsteps; ++i) mpsv::step_species(es, pl->charge, stream);
  });
}

mps_state* mps_plasma_species(mps_plasma* pl, int32_t s) {
  if (!pl || s < 0 || s >= (int32_t)pl->species.size()) return nullptr;
  return pl->species[(size_t)s];
}

mps_status mps_plasma_field(mps_plasma* pl, double* E_out, double* field_energy,
                            hipStream_t stream) {
  return guarded([&] {
    auto es = engines_of(pl);
    mpsv::field_species_dense(es, pl->charge, E_out, field_energy, stream);
  });
}

mps_status mps_plasma_free(mps_plasma* pl) {
  return guarded([&] {
    if (!pl) return;
    (void)hipDeviceSynchronize();
    delete pl;
  });
}
