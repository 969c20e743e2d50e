// MPS engine for the 1D1V Vlasov-Poisson step (Ye & Loureiro,
// arXiv:2205.11990): operators, compression sweep, field solve and RK4.
//
// All device work is enqueued on the caller's stream.  The only host
// synchronisations inside a step are the read-back of each truncated rank
// (the shapes of the following operations depend on it) and the final
// finiteness check that makes a step transactional.
#include <exception>
#include <thread>
#include "engine.hpp"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstdint>
#include <cstring>

#include "gemm.hpp"
#include "mps_kernels.hpp"
#include "prof.hpp"

namespace mpsv {

std::vector<std::pair<int, int>> site_list(int Lx, int Lv, int order) {
  std::vector<std::pair<int, int>> sites;
  if (order == 1 || order == 4) {
    for (int k = 0; k < std::min(Lx, Lv); ++k) {
      sites.push_back({0, k});
      sites.push_back({1, k});
    }
    return sites;
  }
  for (int k = 0; k < Lx; ++k) sites.push_back({0, order == 2 ? Lx - 1 - k : k});
  for (int k = 0; k < Lv; ++k) sites.push_back({1, order == 3 ? Lv - 1 - k : k});
  return sites;
}

// ============================================================ host operators
namespace ops {

namespace {
typedef double M2[2][2];
const M2 I2 = {{1, 0}, {0, 1}};
const M2 SP = {{0, 0}, {1, 0}};  // S+ : (o, i) = (1, 0)
const M2 SM = {{0, 1}, {0, 0}};  // S- : (o, i) = (0, 1)
const M2 P0 = {{1, 0}, {0, 0}};
const M2 P1 = {{0, 0}, {0, 1}};

inline size_t widx(int br, int b, int o, int i, int bp) {
  return ((size_t)(b * 2 + o) * 2 + i) * br + bp;
}
void put(std::vector<double>& W, int br, int b, int bp, const M2& M,
         double sc = 1.0) {
  for (int o = 0; o < 2; ++o)
    for (int i = 0; i < 2; ++i) W[widx(br, b, o, i, bp)] += sc * M[o][i];
}
void put_sum(std::vector<double>& W, int br, int b, int bp, const M2& A,
             const M2& B, double sa, double sb) {
  put(W, br, b, bp, A, sa);
  put(W, br, b, bp, B, sb);
}

// The printed first-derivative MPO (SI, Derivatives): first row, bulk
// matrix, last column.  periodic selects the first-site row.
HostMpo printed_d1(int L, bool periodic, double c1) {
  HostMpo W(L);
  for (int k = 0; k < L; ++k) {
    int bl = (k == 0) ? 1 : 3, br = (k == L - 1) ? 1 : 3;
    W[k].assign((size_t)bl * 4 * br, 0.0);
    if (k == 0) {
      put(W[k], br, 0, 0, I2);
      if (periodic) {
        put_sum(W[k], br, 0, 1, SP, SM, 1, 1);
        put_sum(W[k], br, 0, 2, SP, SM, 1, 1);
      } else {
        put(W[k], br, 0, 1, SM);
        put(W[k], br, 0, 2, SP);
      }
      if (L == 1) throw Error(kEinval, "derivative MPO needs L >= 2");
    } else if (k < L - 1) {
      put(W[k], br, 0, 0, I2);
      put(W[k], br, 0, 1, SM);
      put(W[k], br, 0, 2, SP);
      put(W[k], br, 1, 1, SP);
      put(W[k], br, 2, 2, SM);
    } else {
      put_sum(W[k], br, 0, 0, SM, SP, c1, -c1);
      put(W[k], br, 1, 0, SP, c1);
      put(W[k], br, 2, 0, SM, -c1);
    }
  }
  return W;
}

}  // namespace

HostMpo d1_periodic(int L, double h, std::vector<int>& bonds) {
  HostMpo W = printed_d1(L, true, 0.5);
  // the printed first site already carries bond 1 on the left; if L == 2 the
  // first row meets the last column directly
  for (auto& x : W[0]) x /= h;
  bonds.assign(L + 1, 3);
  bonds[0] = bonds[L] = 1;
  return W;
}

HostMpo d1_zero_gradient(int L, double h, std::vector<int>& bonds) {
  const double c1 = 0.5;
  HostMpo back = printed_d1(L, false, c1);
  // direct sum backbone (3) + M_left (1) + M_right (1): bond 5.
  // M_left  = P0 x ... x P0 x [[0,-c1],[0,0]]   (mirror of the printed M_right)
  // M_right = P1 x ... x P1 x [[0,0],[c1,0]]
  const M2 lastL = {{0, -c1}, {0, 0}};
  const M2 lastR = {{0, 0}, {c1, 0}};
  HostMpo W(L);
  for (int k = 0; k < L; ++k) {
    int bl = (k == 0) ? 1 : 5, br = (k == L - 1) ? 1 : 5;
    W[k].assign((size_t)bl * 4 * br, 0.0);
    int bbl = (k == 0) ? 1 : 3, bbr = (k == L - 1) ? 1 : 3;
    for (int b = 0; b < bbl; ++b)
      for (int bp = 0; bp < bbr; ++bp)
        for (int o = 0; o < 2; ++o)
          for (int i = 0; i < 2; ++i)
            W[k][widx(br, b, o, i, bp)] = back[k][widx(bbr, b, o, i, bp)];
    // extra channels: index 3 (M_left), 4 (M_right) in the middle; on the
    // first site they are columns 3,4; on the last site rows 3,4.
    const bool last = (k == L - 1);
    const M2& ml = last ? lastL : P0;
    const M2& mr = last ? lastR : P1;
    int lrow = (k == 0) ? 0 : 3, rrow = (k == 0) ? 0 : 4;
    int lcol = last ? 0 : 3, rcol = last ? 0 : 4;
    put(W[k], br, lrow, lcol, ml);
    put(W[k], br, rrow, rcol, mr);
  }
  for (auto& x : W[0]) x /= h;
  bonds.assign(L + 1, 5);
  bonds[0] = bonds[L] = 1;
  return W;
}

HostMpo poisson_g(int L, double dx, double scale, std::vector<int>& bonds) {
  // G[o,i] = dx (sign(o-i)/2 - (o-i)/N): comparison automaton over the bit
  // pairs (bond 3: equal / greater / less so far) plus a linear function of
  // the bits (bond 2); direct sum, bond 5.
  if (L < 2) throw Error(kEinval, "Poisson MPO needs L >= 2");
  auto step = [](int s, int o, int i) {
    if (s != 0) return s;
    return o == i ? 0 : (o > i ? 1 : 2);
  };
  const double val[3] = {0.0, 0.5 * dx, -0.5 * dx};
  HostMpo W(L);
  for (int k = 0; k < L; ++k) {
    int bl = (k == 0) ? 1 : 5, br = (k == L - 1) ? 1 : 5;
    W[k].assign((size_t)bl * 4 * br, 0.0);
    const double ck = -dx * std::ldexp(1.0, -1 - k);
    for (int o = 0; o < 2; ++o)
      for (int i = 0; i < 2; ++i) {
        const double d = ck * (double)(o - i);
        if (k == 0) {
          W[k][widx(br, 0, o, i, step(0, o, i))] += 1.0;
          W[k][widx(br, 0, o, i, 3)] += 1.0;
          W[k][widx(br, 0, o, i, 4)] += d;
        } else if (k < L - 1) {
          for (int s = 0; s < 3; ++s) W[k][widx(br, s, o, i, step(s, o, i))] += 1.0;
          W[k][widx(br, 3, o, i, 3)] += 1.0;
          W[k][widx(br, 3, o, i, 4)] += d;
          W[k][widx(br, 4, o, i, 4)] += 1.0;
        } else {
          for (int s = 0; s < 3; ++s) W[k][widx(br, s, o, i, 0)] += val[step(s, o, i)];
          W[k][widx(br, 3, o, i, 0)] += d;
          W[k][widx(br, 4, o, i, 0)] += 1.0;
        }
      }
  }
  for (auto& x : W[0]) x *= scale;
  bonds.assign(L + 1, 5);
  bonds[0] = bonds[L] = 1;
  return W;
}

HostMpo d1_one_sided(int L, double h, bool forward, std::vector<int>& bonds) {
  // (A f)_o = sum_d c_d f_{(o+d) mod N} / h.  Reading the sites from the
  // least significant bit up, the lower bits must reproduce d up to a carry
  // q in {-1, 0, 1}: the last site turns (i - o) into q = (i - o - d) / 2,
  // every other site q_left = (i - o + q_right) / 2; the first site accepts
  // any final carry (periodic wrap).  Bond 3 (state q + 1).
  if (L < 2) throw Error(kEinval, "derivative MPO needs L >= 2");
  const int d[3] = {0, forward ? 1 : -1, forward ? 2 : -2};
  const double c[3] = {forward ? -1.5 : 1.5, forward ? 2.0 : -2.0,
                       forward ? -0.5 : 0.5};
  HostMpo W(L);
  for (int k = 0; k < L; ++k) {
    const int bl = (k == 0) ? 1 : 3, br = (k == L - 1) ? 1 : 3;
    W[k].assign((size_t)bl * 4 * br, 0.0);
    for (int o = 0; o < 2; ++o)
      for (int i = 0; i < 2; ++i) {
        if (k == L - 1) {
          for (int t = 0; t < 3; ++t) {
            const int num = i - o - d[t];
            if (num % 2 != 0) continue;
            const int q = num / 2;
            if (q < -1 || q > 1) continue;
            W[k][widx(br, L == 1 ? 0 : q + 1, o, i, 0)] += c[t];
          }
        } else {
          for (int qr = -1; qr <= 1; ++qr) {
            const int num = i - o + qr;
            if (num % 2 != 0) continue;
            const int ql = num / 2;
            if (k == 0) W[k][widx(br, 0, o, i, qr + 1)] += 1.0;
            else if (ql >= -1 && ql <= 1) W[k][widx(br, ql + 1, o, i, qr + 1)] += 1.0;
          }
        }
      }
  }
  for (auto& x : W[0]) x /= h;
  bonds.assign(L + 1, 3);
  bonds[0] = bonds[L] = 1;
  return W;
}

std::vector<std::vector<double>> poly_mps(int L, double c0, double c1,
                                          double c2, std::vector<int>& bonds) {
  // f(J) = c0 + c1 J + c2 J^2, J = sum_k s_k 2^(L-1-k): carry [1, J, J^2]
  const int deg = (c2 != 0.0) ? 2 : ((c1 != 0.0) ? 1 : 0);
  const int B = deg + 1;
  const double c[3] = {c0, c1, c2};
  std::vector<std::vector<double>> A(L);
  auto T = [&](int s, int k, double* M) {  // B x B
    const double t = s ? std::ldexp(1.0, L - 1 - k) : 0.0;
    for (int a = 0; a < B * B; ++a) M[a] = 0.0;
    for (int a = 0; a < B; ++a) M[a * B + a] = 1.0;
    if (B >= 2) M[0 * B + 1] = t;
    if (B >= 3) {
      M[0 * B + 2] = t * t;
      M[1 * B + 2] = 2.0 * t;
    }
  };
  double M[9];
  for (int k = 0; k < L; ++k) {
    int bl = (k == 0) ? 1 : B, br = (k == L - 1) ? 1 : B;
    A[k].assign((size_t)bl * 2 * br, 0.0);
    for (int s = 0; s < 2; ++s) {
      T(s, k, M);
      for (int a = 0; a < bl; ++a)
        for (int b = 0; b < br; ++b) {
          double v;
          if (k == L - 1) {
            v = 0.0;
            for (int q = 0; q < B; ++q) v += M[a * B + q] * c[q];
            if (L == 1) {  // single site: row 0 only
              v = 0.0;
              for (int q = 0; q < B; ++q) v += M[q] * c[q];
            }
          } else {
            v = M[a * B + b];
          }
          A[k][((size_t)a * 2 + s) * br + b] = v;
        }
    }
  }
  bonds.assign(L + 1, B);
  bonds[0] = bonds[L] = 1;
  return A;
}

HostMpo poly_diag(int L, double c0, double c1, double c2,
                  std::vector<int>& bonds) {
  auto A = poly_mps(L, c0, c1, c2, bonds);
  HostMpo W(L);
  for (int k = 0; k < L; ++k) {
    int bl = bonds[k], br = bonds[k + 1];
    W[k].assign((size_t)bl * 4 * br, 0.0);
    for (int a = 0; a < bl; ++a)
      for (int s = 0; s < 2; ++s)
        for (int b = 0; b < br; ++b)
          W[k][widx(br, a, s, s, b)] = A[k][((size_t)a * 2 + s) * br + b];
  }
  return W;
}

namespace {

// MPS of the indicator of j >= t (ge) or j < t (!ge) over the L bits of j,
// most significant first, 0 < t < 2^L: a comparison with t's bits, states
// "equal so far" and "decided" (bond 2).
std::vector<std::vector<double>> compare_mps(int L, long t, bool ge) {
  std::vector<std::vector<double>> A(L);
  auto bit = [&](int k) { return (int)((t >> (L - 1 - k)) & 1); };
  for (int k = 0; k < L; ++k) {
    const int bl = (k == 0) ? 1 : 2, br = (k == L - 1) ? 1 : 2;
    A[k].assign((size_t)bl * 2 * br, 0.0);
    const int b = bit(k);
    for (int s = 0; s < 2; ++s) {
      const bool decide = ge ? (s > b) : (s < b);
      auto at = [&](int a, int c) -> double& { return A[k][((size_t)a * 2 + s) * br + c]; };
      if (k == L - 1) {
        at(0, 0) = (decide || (ge && s == b)) ? 1.0 : 0.0;
        if (bl == 2) at(1, 0) = 1.0;
      } else {
        at(0, 0) = (s == b) ? 1.0 : 0.0;
        at(0, 1) = decide ? 1.0 : 0.0;
        if (bl == 2) at(1, 1) = 1.0;
      }
    }
  }
  return A;
}

// Elementwise product of two MPS (bonds multiply).
std::vector<std::vector<double>> hadamard(
    const std::vector<std::vector<double>>& A, const std::vector<int>& ba,
    const std::vector<std::vector<double>>& B, const std::vector<int>& bb,
    std::vector<int>& bonds) {
  const int L = (int)A.size();
  std::vector<std::vector<double>> C(L);
  bonds.assign(L + 1, 1);
  for (int k = 0; k <= L; ++k) bonds[k] = ba[k] * bb[k];
  for (int k = 0; k < L; ++k) {
    const int al = ba[k], ar = ba[k + 1], cl = bb[k], cr = bb[k + 1];
    C[k].assign((size_t)al * cl * 2 * ar * cr, 0.0);
    for (int a = 0; a < al; ++a)
      for (int c = 0; c < cl; ++c)
        for (int s = 0; s < 2; ++s)
          for (int b = 0; b < ar; ++b)
            for (int e = 0; e < cr; ++e)
              C[k][(((size_t)(a * cl + c) * 2 + s) * ar + b) * cr + e] =
                  A[k][((size_t)a * 2 + s) * ar + b] * B[k][((size_t)c * 2 + s) * cr + e];
  }
  return C;
}

}  // namespace

HostMpo velocity_part_diag(int L, double v0, double dv, bool positive,
                           std::vector<int>& bonds) {
  // max(v_j, 0) = v_j [j >= j0], min(v_j, 0) = v_j [j < j1]
  const long N = 1L << L;
  auto v = [&](long j) { return v0 + (double)j * dv; };
  long t = 0;
  if (positive) {
    while (t < N && v(t) <= 0.0) ++t;  // first j with v_j > 0
  } else {
    while (t < N && v(t) < 0.0) ++t;   // first j with v_j >= 0
  }
  const bool empty = positive ? (t >= N) : (t == 0);
  const bool full = positive ? (t == 0) : (t >= N);
  std::vector<int> bp;
  auto P = poly_mps(L, v0, dv, 0.0, bp);
  std::vector<std::vector<double>> A;
  if (empty) {
    bonds.assign(L + 1, 1);
    A.assign(L, std::vector<double>(2, 0.0));
  } else if (full) {
    A = P;
    bonds = bp;
  } else {
    std::vector<int> bc(L + 1, 2);
    bc[0] = bc[L] = 1;
    A = hadamard(P, bp, compare_mps(L, t, positive), bc, bonds);
  }
  HostMpo W(L);
  for (int k = 0; k < L; ++k) {
    const int bl = bonds[k], br = bonds[k + 1];
    W[k].assign((size_t)bl * 4 * br, 0.0);
    for (int a = 0; a < bl; ++a)
      for (int s = 0; s < 2; ++s)
        for (int b = 0; b < br; ++b)
          W[k][widx(br, a, s, s, b)] = A[k][((size_t)a * 2 + s) * br + b];
  }
  return W;
}

HostMpo mpo_add(const HostMpo& A, const std::vector<int>& ba, const HostMpo& B,
                const std::vector<int>& bb, std::vector<int>& bonds) {
  const int L = (int)A.size();
  if (L < 2 || (int)B.size() != L) throw Error(kEinval, "mpo_add: bad lengths");
  bonds.assign(L + 1, 1);
  for (int k = 1; k < L; ++k) bonds[k] = ba[k] + bb[k];
  HostMpo W(L);
  for (int k = 0; k < L; ++k) {
    const int bl = bonds[k], br = bonds[k + 1];
    W[k].assign((size_t)bl * 4 * br, 0.0);
    // block offsets of A and B in the left / right bonds
    const int al = ba[k], ar = ba[k + 1], cl = bb[k], cr = bb[k + 1];
    const int offBl = (k == 0) ? 0 : al, offBr = (k == L - 1) ? 0 : ar;
    for (int a = 0; a < al; ++a)
      for (int o = 0; o < 2; ++o)
        for (int i = 0; i < 2; ++i)
          for (int b = 0; b < ar; ++b)
            W[k][widx(br, a, o, i, b)] += A[k][widx(ar, a, o, i, b)];
    for (int a = 0; a < cl; ++a)
      for (int o = 0; o < 2; ++o)
        for (int i = 0; i < 2; ++i)
          for (int b = 0; b < cr; ++b)
            W[k][widx(br, offBl + a, o, i, offBr + b)] += B[k][widx(cr, a, o, i, b)];
  }
  return W;
}

HostMpo mpo_product(const HostMpo& A, const std::vector<int>& ba,
                    const HostMpo& B, const std::vector<int>& bb,
                    std::vector<int>& bonds) {
  const int L = (int)A.size();
  if ((int)B.size() != L) throw Error(kEinval, "mpo_product: bad lengths");
  bonds.assign(L + 1, 1);
  for (int k = 0; k <= L; ++k) bonds[k] = ba[k] * bb[k];
  HostMpo W(L);
  for (int k = 0; k < L; ++k) {
    const int al = ba[k], ar = ba[k + 1], cl = bb[k], cr = bb[k + 1];
    const int br = ar * cr;
    W[k].assign((size_t)al * cl * 4 * br, 0.0);
    for (int a = 0; a < al; ++a)
      for (int c = 0; c < cl; ++c)
        for (int o = 0; o < 2; ++o)
          for (int i = 0; i < 2; ++i)
            for (int b = 0; b < ar; ++b)
              for (int d = 0; d < cr; ++d) {
                double t = 0.0;
                for (int m = 0; m < 2; ++m)
                  t += A[k][widx(ar, a, o, m, b)] * B[k][widx(cr, c, m, i, d)];
                W[k][widx(br, a * cl + c, o, i, b * cr + d)] = t;
              }
  }
  return W;
}

// Full-chain tensor for P physical values per site (4: MPO, 2: MPS).  A
// dimension read fine to coarse (S2: x, S3: v) takes its cores in reverse
// order with their two bonds swapped.
static HostMpo chain_generic(const HostMpo& Wx, const std::vector<int>& bx,
                             const HostMpo& Wv, const std::vector<int>& bv,
                             int order, int P, std::vector<int>& bonds) {
  const int Lx = (int)Wx.size(), Lv = (int)Wv.size();
  if ((order == 1 || order == 4) && Lx != Lv)
    throw Error(kEinval, "interleaved ordering needs Lx == Lv");
  const auto sites = site_list(Lx, Lv, order);
  HostMpo out;
  bonds.assign(1, 1);
  int cx = 1, cv = 1;
  for (auto& st : sites) {
    const int k = st.second;
    const bool isx = st.first == 0;
    const bool rev = isx ? order == 2 : order == 3;
    const std::vector<double>& W = isx ? Wx[k] : Wv[k];
    const std::vector<int>& bd = isx ? bx : bv;
    const int l0 = bd[k], r0 = bd[k + 1];
    const int l = rev ? r0 : l0, r = rev ? l0 : r0;
    auto val = [&](int a, int p, int b) {
      return rev ? W[((size_t)b * P + p) * r0 + a] : W[((size_t)a * P + p) * r0 + b];
    };
    if (isx) {
      const int d = cv;
      std::vector<double> T((size_t)l * d * P * r * d, 0.0);
      for (int a = 0; a < l; ++a)
        for (int c = 0; c < d; ++c)
          for (int p = 0; p < P; ++p)
            for (int b = 0; b < r; ++b)
              T[(((size_t)(a * d + c) * P + p) * r + b) * d + c] = val(a, p, b);
      out.push_back(std::move(T));
      bonds.push_back(r * d);
      cx = r;
    } else {
      const int d = cx;
      std::vector<double> T((size_t)d * l * P * d * r, 0.0);
      for (int c = 0; c < d; ++c)
        for (int a = 0; a < l; ++a)
          for (int p = 0; p < P; ++p)
            for (int b = 0; b < r; ++b)
              T[(((size_t)(c * l + a) * P + p) * d + c) * r + b] = val(a, p, b);
      out.push_back(std::move(T));
      bonds.push_back(d * r);
      cv = r;
    }
  }
  return out;
}

HostMpo reverse(const HostMpo& W, const std::vector<int>& bonds, int P,
                std::vector<int>& out_bonds) {
  const int L = (int)W.size();
  HostMpo out(L);
  out_bonds.assign(L + 1, 1);
  for (int j = 0; j < L; ++j) {
    const int k = L - 1 - j;
    const int l0 = bonds[k], r0 = bonds[k + 1];
    out[j].assign(W[k].size(), 0.0);
    for (int a = 0; a < l0; ++a)
      for (int p = 0; p < P; ++p)
        for (int b = 0; b < r0; ++b)
          out[j][((size_t)b * P + p) * l0 + a] = W[k][((size_t)a * P + p) * r0 + b];
    out_bonds[j] = r0;
    out_bonds[j + 1] = l0;
  }
  return out;
}

HostMpo chain(const HostMpo& Wx, const std::vector<int>& bx, const HostMpo& Wv,
              const std::vector<int>& bv, int order, std::vector<int>& bonds) {
  return chain_generic(Wx, bx, Wv, bv, order, 4, bonds);
}

HostMpo chain_mps(const HostMpo& Ax, const std::vector<int>& bx,
                  const HostMpo& Av, const std::vector<int>& bv, int order,
                  std::vector<int>& bonds) {
  return chain_generic(Ax, bx, Av, bv, order, 2, bonds);
}

}  // namespace ops

// ================================================================= engine

static int cap_or_inf(int c) { return c > 0 ? c : INT_MAX; }

MemoryModel memory_model(const Problem& q) {
  const int n = q.n();
  const double chi = q.chi_max;
  auto full = [&](int j) { return std::ldexp(1.0, std::min(j, n - j)); };
  // field bond: the cap D_F, at most the full rank of an Lx-site MPS
  const double df = std::min(q.df_max > 0 ? (double)q.df_max : chi,
                             std::ldexp(1.0, q.Lx / 2));
  // widest MPO of each lane.  Main lane: the field term, and with the
  // moment collision model the temperature term diag(vth^2) (x) Dv Dv (the
  // temperature capped like the field: bond 25 D_F in the interleaved
  // order).  Side lane: the advection term (central or upwind) and the
  // fixed collision operator nu Dv (diag(v - v0) + vth^2 Dv) (bond 35 on
  // the v sites) or the moment model's nu Dv diag(v) (bond 10).
  const bool il = q.order == 1 || q.order == 4;
  double wm = (il ? 5.0 : 3.0) * df;
  double ws = q.x_scheme == 1 ? (il ? 24.0 : 8.0) : (il ? 6.0 : 3.0);
  if (q.nu != 0.0) {
    if (q.coll_model == 1) {
      ws = std::max(ws, 35.0);
    } else {
      wm = std::max(wm, il ? 25.0 * df : std::max(25.0, df));
      ws = std::max(ws, 10.0);
    }
  }
  // bond cap at bond j: chi, or 2 chi inside an IG pair (never cut there)
  auto cap = [&](int j) { return (q.order == 4 && (j & 1)) ? 2.0 * chi : chi; };
  double S = 0, N = 0, Ns = 0, I = 0;
  for (int j = 0; j < n; ++j) {
    const double bl = std::min(cap(j), full(j)), br = std::min(cap(j + 1), full(j + 1));
    S += bl * 2 * br;
    N = std::max(N, std::min(wm * bl, full(j)) * wm * 2 * br);
    Ns = std::max(Ns, std::min(ws * bl, full(j)) * ws * 2 * br);
  }
  if (il) {
    // interleaved initial state: Kronecker products of the x and v cores
    // of the profiles' iterated SVDs, whose ranks are taken as at most 32
    // (smooth profiles keep a handful of values above the 1e-14 cut)
    auto fr = [&](int k) { return std::min(32.0, std::ldexp(1.0, std::min(k, q.Lx - k))); };
    for (int k = 0; k < q.Lx; ++k)
      I += fr(k) * fr(k) * 2 * fr(k + 1) * fr(k) +
           fr(k) * fr(k + 1) * 2 * fr(k + 1) * fr(k + 1);
  }
  S *= 8.0;
  N *= 8.0;
  Ns *= 8.0;
  // compact-WY mode: a 64 x 64 T beside each group of 64 reflectors of a
  // block over 512 rows (under 1/7 of the group's reflector storage)
  if (q.tall_apply == 1) {
    N *= 1.15;
    Ns *= 1.15;
  }
  I *= 8.0;
  double work = il ? std::max({12.0 * N, 3.5 * I, 60.0 * S}) : std::max(60.0 * S, 12.0 * N);
  double work2 = std::max(80.0 * S, 12.0 * Ns);
  // centre-first: the right half's sweep holds its own blocks beside
  if (q.compression == 1) {
    work += 20.0 * S;
    work2 += 20.0 * S;
  }
  const double est[7] = {1.0 * (1 << 20), 2.0 * S, 1.5 * I + 12.0 * S, 40.0 * S,
                         work, 40.0 * S, work2};
  MemoryModel m;
  m.chunk = (size_t)std::min(64.0 * (1 << 20), std::max(2.0 * (1 << 20), 8.0 * S));
  m.chunk = (m.chunk + 255) & ~(size_t)255;
  m.bound = (size_t)32 << 20;
  for (int i = 0; i < 7; ++i) {
    m.arena[i] = (size_t)est[i];
    m.bound += m.arena[i] + 2 * m.chunk;
  }
  return m;
}

size_t Engine::device_bytes() const {
  return ops_.reserved_bytes() + state_.reserved_bytes() + step_.reserved_bytes() +
         tmp_.reserved_bytes() + work_.reserved_bytes() + tmp2_.reserved_bytes() +
         work2_.reserved_bytes();
}

void Engine::arena_bytes(size_t reserved[7], size_t peak[7]) const {
  const Arena* a[7] = {&ops_, &state_, &step_, &tmp_, &work_, &tmp2_, &work2_};
  for (int i = 0; i < 7; ++i) {
    reserved[i] = a[i]->reserved_bytes();
    peak[i] = a[i]->peak_bytes();
  }
}

// Parameter checks of a problem (host only; shared by state creation and
// the admission bound).
void validate_problem(const Problem& p) {
  MPSV_CHECK(p.Lx >= 2 && p.Lx <= 14 && p.Lv >= 2 && p.Lv <= 14, kEinval,
             "Lx and Lv must lie in [2, 14]");
  MPSV_CHECK(p.order >= 0 && p.order <= 4, kEinval, "unknown ordering");
  MPSV_CHECK((p.order != 1 && p.order != 4) || p.Lx == p.Lv, kEinval,
             "interleaved ordering needs Lx == Lv");
  MPSV_CHECK(p.x_max > p.x_min && p.v_max > p.v_min, kEinval,
             "empty x or v interval");
  MPSV_CHECK(std::isfinite(p.cfl) && p.cfl >= 0, kEinval, "cfl must be >= 0");
  MPSV_CHECK(p.cfl > 0 || (std::isfinite(p.dt) && p.dt > 0), kEinval,
             "dt must be > 0");
  MPSV_CHECK(p.chi_max >= 1, kEinval, "chi_max must be >= 1");
  MPSV_CHECK(p.level >= 1 && p.level <= 5, kEinval, "level must be in 1..5");
  MPSV_CHECK(p.df_max >= 0, kEinval, "df_max must be >= 0");
  MPSV_CHECK(std::isfinite(p.tol) && p.tol >= 0, kEinval, "tol must be >= 0");
  MPSV_CHECK(p.precision >= 0 && p.precision <= 2, kEinval,
             "unknown precision mode");
  MPSV_CHECK(p.x_scheme == 0 || p.x_scheme == 1, kEinval,
             "unknown x advection scheme");
  MPSV_CHECK(std::isfinite(p.qm), kEinval, "q/m must be finite");
  MPSV_CHECK(std::isfinite(p.nu) && p.nu >= 0 && std::isfinite(p.nu_v0) &&
                 std::isfinite(p.nu_vth),
             kEinval, "collision parameters must be finite, nu >= 0");
  MPSV_CHECK(p.coll_model == 0 || p.coll_model == 1, kEinval,
             "unknown collision model");
  MPSV_CHECK(p.tall_apply == 0 || p.tall_apply == 1, kEinval,
             "unknown reflector application mode");
  MPSV_CHECK(p.compression == 0 || p.compression == 1, kEinval,
             "unknown compression scheme");
  MPSV_CHECK(p.compression == 0 || (p.order != 1 && p.order != 4), kEinval,
             "centre-first compression needs a sequential ordering");
}

namespace {

// The host-built operators of one problem (exact, FP64).
struct HostOps {
  ops::HostMpo T1, G, coll, Dv, Dv2;
  std::vector<int> bt1, bg, bcoll, bdv, bdv2;
  std::vector<std::vector<double>> vpoly, v2poly;
  std::vector<int> bpoly, bpoly2;
};

HostOps host_operators(const Problem& p) {
  HostOps h;
  if (p.x_scheme == 1) {
    // upwind: T1 = -(Db (x) diag(max(v,0)) + Df (x) diag(min(v,0))) f
    std::vector<int> bdb, bdf, bvp, bvn, btp, btn;
    auto Db = ops::d1_one_sided(p.Lx, p.dx(), false, bdb);
    auto Df = ops::d1_one_sided(p.Lx, p.dx(), true, bdf);
    auto Vp = ops::velocity_part_diag(p.Lv, p.v_min, p.dv(), true, bvp);
    auto Vn = ops::velocity_part_diag(p.Lv, p.v_min, p.dv(), false, bvn);
    auto Tp = ops::chain(Db, bdb, Vp, bvp, p.order, btp);
    auto Tn = ops::chain(Df, bdf, Vn, bvn, p.order, btn);
    h.T1 = ops::mpo_add(Tp, btp, Tn, btn, h.bt1);
  } else {
    std::vector<int> bdx, bvv;
    auto Dx = ops::d1_periodic(p.Lx, p.dx(), bdx);
    auto V = ops::poly_diag(p.Lv, p.v_min, p.dv(), 0.0, bvv);
    h.T1 = ops::chain(Dx, bdx, V, bvv, p.order, h.bt1);
  }
  for (auto& x : h.T1[0]) x = -x;  // T1 = -(advection) f
  h.G = ops::poisson_g(p.Lx, p.dx(), -1.0, h.bg);  // E = -G n
  if (p.nu != 0.0) {
    // Dougherty collisions (Methods, Collision Operator) on the v sites, the
    // identity on the x sites
    std::vector<int> bd, bpd, bcv;
    auto D1 = ops::d1_zero_gradient(p.Lv, p.dv(), bd);
    ops::HostMpo Cv;
    if (p.coll_model == 1) {
      // the species' fixed drift and thermal speed: nu Dv (diag(v - v0) +
      // vth^2 Dv)
      std::vector<int> bin;
      auto Vd = ops::poly_diag(p.Lv, p.v_min - p.nu_v0, p.dv(), 0.0, bpd);
      auto Ds = D1;
      for (auto& x : Ds[0]) x *= p.nu_vth * p.nu_vth;
      auto inner = ops::mpo_add(Vd, bpd, Ds, bd, bin);
      Cv = ops::mpo_product(D1, bd, inner, bin, bcv);
    } else {
      // the moments of f: nu Dv diag(v) is fixed; the drift and temperature
      // terms are built per stage, the latter with Dv Dv
      auto Vd = ops::poly_diag(p.Lv, p.v_min, p.dv(), 0.0, bpd);
      Cv = ops::mpo_product(D1, bd, Vd, bpd, bcv);
      h.Dv2 = ops::mpo_product(D1, bd, D1, bd, h.bdv2);
      if (p.order == 3) {
        std::vector<int> brev;
        h.Dv2 = ops::reverse(h.Dv2, h.bdv2, 4, brev);
        h.bdv2 = brev;
      }
    }
    for (auto& x : Cv[0]) x *= p.nu;
    ops::HostMpo Ix((size_t)p.Lx, std::vector<double>{1.0, 0.0, 0.0, 1.0});
    std::vector<int> bix((size_t)p.Lx + 1, 1);
    h.coll = ops::chain(Ix, bix, Cv, bcv, p.order, h.bcoll);
  }
  h.Dv = ops::d1_zero_gradient(p.Lv, p.dv(), h.bdv);
  if (p.order == 3) {
    // v read fine to coarse (S3): Dv in chain order
    std::vector<int> brev;
    h.Dv = ops::reverse(h.Dv, h.bdv, 4, brev);
    h.bdv = brev;
  }
  // moment weights 1(x) w(v), w = v, v^2/2 as full-chain MPS
  std::vector<int> b1, bw, bw2;
  auto onesx = ops::poly_mps(p.Lx, 1.0, 0.0, 0.0, b1);
  auto wv = ops::poly_mps(p.Lv, p.v_min, p.dv(), 0.0, bw);
  h.vpoly = ops::chain_mps(onesx, b1, wv, bw, p.order, h.bpoly);
  auto wv2 = ops::poly_mps(p.Lv, 0.5 * p.v_min * p.v_min, p.v_min * p.dv(),
                           0.5 * p.dv() * p.dv(), bw2);
  h.v2poly = ops::chain_mps(onesx, b1, wv2, bw2, p.order, h.bpoly2);
  return h;
}

// Parameter checks of a batch of lock-step instances: one shape, one time
// step, fixed ranks.
void validate_batch(const std::vector<Problem>& ps) {
  MPSV_CHECK(!ps.empty(), kEinval, "a batch needs at least one instance");
  for (auto& q : ps) validate_problem(q);
  if (ps.size() == 1) return;
  const Problem& a = ps[0];
  for (auto& b : ps) {
    MPSV_CHECK(b.Lx == a.Lx && b.Lv == a.Lv && b.order == a.order &&
                   b.chi_max == a.chi_max && b.level == a.level &&
                   b.df_max == a.df_max && b.precision == a.precision &&
                   b.x_scheme == a.x_scheme && b.compression == a.compression &&
                   b.tall_apply == a.tall_apply,
               kEinval, "lock-step instances must share the problem shape");
    MPSV_CHECK(b.tol == 0.0 && b.cfl == 0.0 && b.dt == a.dt && b.qm == a.qm,
               kEinval,
               "lock-step instances need tol = 0, a fixed and common dt and q/m");
    MPSV_CHECK((b.nu != 0.0) == (a.nu != 0.0) && b.coll_model == a.coll_model, kEinval,
               "lock-step instances are all collisionless or all of one collision model");
  }
}

// Arena chunk of a batch: every single request must fit one chunk (the
// widest MPO x MPS contraction of the field term dominates).
size_t batch_chunk(const Problem& p, int n) {
  const MemoryModel m = memory_model(p);
  if (n == 1) return m.chunk;
  const int L = p.n();
  const double chi = p.chi_max;
  const double df = std::min(p.df_max > 0 ? (double)p.df_max : chi,
                             std::ldexp(1.0, p.Lx / 2));
  const bool il = p.order == 1 || p.order == 4;
  const double w = std::max((il ? 5.0 : 3.0) * df, p.x_scheme == 1 ? 24.0 : 6.0);
  double big = 0;
  for (int j = 0; j <= L; ++j) {
    const double full = std::ldexp(1.0, std::min(j, L - j));
    const double b = std::min(chi, full);
    big = std::max(big, std::min(w * b, std::ldexp(1.0, std::min(j, 30))) * w * 2 * b);
  }
  size_t c = (size_t)(8.0 * big * 1.25) + ((size_t)1 << 20);
  c = std::max(c, m.chunk);
  c = std::max(c, (size_t)64 << 20);
  return (c + 255) & ~(size_t)255;
}

}  // namespace

Engine::Engine(const Problem& p) : Engine(std::vector<Problem>{p}) {}

// (the checks run before the size model reads the problem)
Engine::Engine(const std::vector<Problem>& batch)
    : p_((validate_batch(batch), batch[0])), ps_(batch), nin_((int)batch.size()),
      chunk_(batch_chunk(batch[0], (int)batch.size())) {
  MPSV_HIP(hipGetDevice(&device_));
  MPSV_HIP(hipStreamCreateWithFlags(&own_, hipStreamNonBlocking));
  MPSV_HIP(hipStreamCreateWithFlags(&side_, hipStreamNonBlocking));
  MPSV_HIP(hipEventCreateWithFlags(&ev_fork_, hipEventDisableTiming));
  MPSV_HIP(hipEventCreateWithFlags(&ev_join_, hipEventDisableTiming));
  MPSV_HIP(hipEventCreateWithFlags(&ev_in_, hipEventDisableTiming));
  MPSV_HIP(hipEventCreateWithFlags(&ev_out_, hipEventDisableTiming));
  LanesScope ls(all_lanes());

  hipStream_t s = nullptr;
  std::vector<HostOps> h;
  for (auto& q : ps_) h.push_back(host_operators(q));
  for (auto& x : h)
    MPSV_CHECK(x.bt1 == h[0].bt1 && x.bg == h[0].bg && x.bcoll == h[0].bcoll &&
                   x.bdv == h[0].bdv && x.bdv2 == h[0].bdv2 && x.bpoly == h[0].bpoly &&
                   x.bpoly2 == h[0].bpoly2,
               kEinval, "lock-step instances need operators of the same bonds");
  auto pick = [&](ops::HostMpo HostOps::*m) {
    std::vector<const ops::HostMpo*> v;
    for (auto& x : h) v.push_back(&(x.*m));
    return v;
  };
  t1_ = upload_mpo(pick(&HostOps::T1), h[0].bt1, ops_, s);
  gneg_ = upload_mpo(pick(&HostOps::G), h[0].bg, ops_, s);
  if (p_.nu != 0.0) coll_ = upload_mpo(pick(&HostOps::coll), h[0].bcoll, ops_, s);
  if (p_.nu != 0.0 && p_.coll_model == 0)
    dv2_ = upload_mpo(pick(&HostOps::Dv2), h[0].bdv2, ops_, s);
  dv_ = upload_mpo(pick(&HostOps::Dv), h[0].bdv, ops_, s);
  auto upload_chain = [&](std::vector<std::vector<double>> HostOps::*m,
                          const std::vector<int>& bc) {
    DMps out((h[0].*m).size());
    for (size_t j = 0; j < out.size(); ++j) {
      out[j].l = bc[j];
      out[j].r = bc[j + 1];
      out[j].p = ops_.alloc((h[0].*m)[j].size());
      for (int i = 0; i < nin_; ++i)
        MPSV_HIP(hipMemcpy(shifted(out[j].p, (long)i * (long)chunk_),
                           (h[i].*m)[j].data(), (h[i].*m)[j].size() * sizeof(double),
                           hipMemcpyHostToDevice));
    }
    return out;
  };
  vpoly_ = upload_chain(&HostOps::vpoly, h[0].bpoly);
  v2poly_ = upload_chain(&HostOps::v2poly, h[0].bpoly2);
  dflag_ = ops_.alloc_int(4);
  ident_ = ops_.alloc((size_t)kIdent * kIdent);
  identity(s, ident_, kIdent);
  out_main_.bind(ops_.alloc((size_t)SvdOutcomes::kSlots * SvdOutcomes::kInfoWords));
  out_side_.bind(ops_.alloc((size_t)SvdOutcomes::kSlots * SvdOutcomes::kInfoWords));
  disc_.assign((size_t)(n() - 1) * nin_, 0.0);
  MPSV_HIP(hipDeviceSynchronize());
}

void Engine::check_instance(int i) const {
  MPSV_CHECK(i >= 0 && i < nin_, kEinval, "instance index out of range");
}

std::vector<double> Engine::last_discarded(int inst) const {
  check_instance(inst);
  std::vector<double> d((size_t)n() - 1, 0.0);
  const size_t off = (size_t)inst * (size_t)(n() - 1);
  for (size_t j = 0; j < d.size() && off + j < disc_.size(); ++j) d[j] = disc_[off + j];
  return d;
}

Engine::~Engine() {
  // the side stream may still read buffers owned by the arenas
  if (side_) (void)hipStreamSynchronize(side_);
  if (own_) (void)hipStreamSynchronize(own_);
  if (gexec_) (void)hipGraphExecDestroy(gexec_);
  if (ev_fork_) (void)hipEventDestroy(ev_fork_);
  if (ev_join_) (void)hipEventDestroy(ev_join_);
  if (ev_in_) (void)hipEventDestroy(ev_in_);
  if (ev_out_) (void)hipEventDestroy(ev_out_);
  if (side_) (void)hipStreamDestroy(side_);
  if (own_) (void)hipStreamDestroy(own_);
}

namespace {
// Set on the side thread of Engine::rhs for its duration.
thread_local Arena* tl_work = nullptr;
}  // namespace

Arena& Engine::work() { return tl_work ? *tl_work : work_; }

namespace {
// Host <-> device copies of the one instance the calling thread's lanes
// cover: the device side is shifted to that instance.
void d2h(hipStream_t s, void* h, const void* d, size_t bytes) {
  MPSV_CHECK(inst_count() == 1, kEinval, "a read-back covers one instance");
  MPSV_HIP(hipMemcpyAsync(h, shifted(d, lanes().first), bytes,
                          hipMemcpyDeviceToHost, s));
}
void d2d_out(hipStream_t s, void* dst, const void* src, size_t bytes) {
  MPSV_CHECK(inst_count() == 1, kEinval, "a copy out covers one instance");
  MPSV_HIP(hipMemcpyAsync(dst, shifted(src, lanes().first), bytes,
                          hipMemcpyDeviceToDevice, s));
}
void d2d_in(hipStream_t s, void* dst, const void* src, size_t bytes) {
  MPSV_CHECK(inst_count() == 1, kEinval, "a copy in covers one instance");
  MPSV_HIP(hipMemcpyAsync(shifted(dst, lanes().first), src, bytes,
                          hipMemcpyDeviceToDevice, s));
}
// A caller's device buffer handed to a kernel under the lanes of one
// instance: kernels shift every pointer to their instance, so the caller's
// pointer enters with that shift taken off.
template <class T>
T* foreign(T* p) {
  return reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(p) - (uintptr_t)lanes().first);
}
}  // namespace

DMpo Engine::upload_mpo(const std::vector<std::vector<double>>& W,
                        const std::vector<int>& bonds, Arena& ar,
                        hipStream_t s) {
  LanesScope ls(one_lane(0));
  return upload_mpo(std::vector<const ops::HostMpo*>{&W}, bonds, ar, s);
}

// One MPO per instance of the calling thread's lanes (same bonds).
DMpo Engine::upload_mpo(const std::vector<const ops::HostMpo*>& Ws,
                        const std::vector<int>& bonds, Arena& ar,
                        hipStream_t s) {
  MPSV_CHECK((int)Ws.size() == inst_count(), kEinval,
             "one MPO per instance expected");
  const ops::HostMpo& W = *Ws[0];
  DMpo out(W.size());
  for (size_t j = 0; j < W.size(); ++j) {
    MpoSite& m = out[j];
    m.wl = bonds[j];
    m.wr = bonds[j + 1];
    m.W = ar.alloc(W[j].size());
    m.Wmat = ar.alloc(W[j].size());
    for (size_t i = 0; i < Ws.size(); ++i) {
      const auto& Wi = (*Ws[i])[j];
      MPSV_CHECK((long)Wi.size() == (long)m.wl * 4 * m.wr, kEinval,
                 "MPO site size mismatch");
      MPSV_HIP(hipMemcpy(shifted(m.W, lanes().first + (long)i * lanes().stride),
                         Wi.data(), Wi.size() * sizeof(double),
                         hipMemcpyHostToDevice));
    }
    mpo_left_matrix(s, m.W, m.wl, m.wr, m.Wmat);
  }
  return out;
}

int Engine::cap_for(int point) const {
  return (p_.level >= point) ? cap_or_inf(p_.chi_max) : INT_MAX;
}

std::vector<int> Engine::bonds() const {
  std::vector<int> b(n() + 1, 1);
  for (int j = 0; j < (int)f_.size(); ++j) b[j + 1] = f_[j].r;
  if (!f_.empty()) b[0] = f_[0].l;
  return b;
}

// M (p x 2 x v.r) = R (p x v.l, contiguous) * C_j
void Engine::absorb_left(const VSite& v, const double* R, int p, double* M,
                         hipStream_t s) {
  switch (v.kind) {
    case VSite::kDense: {
      gemm(s, p, 2 * v.r, v.l, 1.0, CMatView{R, v.l, 1, 0},
           CMatView{v.A.p, 2L * v.r, 1, 0}, 0.0, MatView{M, 2L * v.r, 1, 0}, 1, 0,
           &work());
      break;
    }
    case VSite::kApply: {
      const int wl = v.W.wl, wr = v.W.wr, al = v.A.l, ar = v.A.r;
      ArenaScope sc(work());
      double* X = work().alloc((size_t)p * wl * 2 * ar);
      // X[(p,b)][(i,a')] = sum_a R[p][(b,a)] A[a][i][a']
      gemm(s, p * wl, 2 * ar, al, 1.0, CMatView{R, al, 1, 0},
           CMatView{v.A.p, 2L * ar, 1, 0}, 0.0, MatView{X, 2L * ar, 1, 0}, 1,
           contract_prec(), &work());
      // M_p[(o,b')][a'] = sum_(b,i) Wmat[(o,b')][(b,i)] X_p[(b,i)][a']
      gemm(s, 2 * wr, ar, 2 * wl, 1.0, CMatView{v.W.Wmat, 2L * wl, 1, 0},
           CMatView{X, ar, 1, 2L * wl * ar}, 0.0,
           MatView{M, ar, 1, 2L * wr * ar}, p, contract_prec());
      break;
    }
    case VSite::kSum: {
      const int T = (int)v.terms.size();
      for (int t = 0; t < T; ++t) {
        const Core& A = v.terms[t];
        if (v.pos == 0) {
          // M[p][s][roff+b] = coef * R[p][0] * A[0][s][b]
          gemm(s, p, A.r, 1, v.coef[t], CMatView{R, 1, 1, 0},
               CMatView{A.p, 2L * A.r, 1, A.r}, 0.0,
               MatView{M + v.roff[t], 2L * v.r, 1, v.r}, 2);
        } else if (v.pos == 1) {
          gemm(s, p, A.r, A.l, 1.0, CMatView{R + v.loff[t], v.l, 1, 0},
               CMatView{A.p, 2L * A.r, 1, A.r}, 0.0,
               MatView{M + v.roff[t], 2L * v.r, 1, v.r}, 2);
        } else {
          gemm(s, p, 2, A.l, 1.0, CMatView{R + v.loff[t], v.l, 1, 0},
               CMatView{A.p, 2, 1, 0}, t == 0 ? 0.0 : 1.0,
               MatView{M, 2, 1, 0});
        }
      }
      break;
    }
    case VSite::kCopy: {
      // natural-basis isometry: (p x l) with l = 2 r is already p x 2 x r
      copy_doubles(s, M, R, (long)p * v.l);
      break;
    }
  }
}

// N (v.l x 2 x q) = C_j * L (v.r x q, contiguous)
void Engine::absorb_right(const VSite& v, const double* L, int q, double* N,
                          hipStream_t s) {
  switch (v.kind) {
    case VSite::kDense: {
      gemm(s, 2 * v.l, q, v.r, 1.0, CMatView{v.A.p, v.r, 1, 0},
           CMatView{L, q, 1, 0}, 0.0, MatView{N, q, 1, 0}, 1, 0, &work());
      break;
    }
    case VSite::kApply: {
      const int wl = v.W.wl, wr = v.W.wr, al = v.A.l, ar = v.A.r;
      ArenaScope sc(work());
      // Z[(a,i)][b'][q] = sum_a' A[a][i][a'] L[(b',a')][q]   (batch b')
      double* Z = work().alloc((size_t)al * 2 * wr * q);
      gemm(s, 2 * al, q, ar, 1.0, CMatView{v.A.p, ar, 1, 0},
           CMatView{L, q, 1, (long)ar * q}, 0.0,
           MatView{Z, (long)wr * q, 1, q}, wr, contract_prec());
      // N'[a][(b,o)][q] = sum_(i,b') W[(b,o)][(i,b')] Z[a][(i,b')][q]
      double* Np = work().alloc((size_t)al * wl * 2 * q);
      gemm(s, 2 * wl, q, 2 * wr, 1.0, CMatView{v.W.W, 2L * wr, 1, 0},
           CMatView{Z, q, 1, 2L * wr * q}, 0.0,
           MatView{Np, q, 1, 2L * wl * q}, al, contract_prec());
      // N[b][a][o][q] = N'[a][b][o][q]
      swap01(s, Np, al, wl, 2L * q, N);
      break;
    }
    case VSite::kSum: {
      const int T = (int)v.terms.size();
      for (int t = 0; t < T; ++t) {
        const Core& A = v.terms[t];
        const double* Lt = (v.pos == 2) ? L : L + (long)v.roff[t] * q;
        if (v.pos == 0) {
          gemm(s, 2, q, A.r, v.coef[t], CMatView{A.p, A.r, 1, 0},
               CMatView{Lt, q, 1, 0}, t == 0 ? 0.0 : 1.0,
               MatView{N, q, 1, 0});
        } else {
          gemm(s, 2 * A.l, q, A.r, 1.0, CMatView{A.p, A.r, 1, 0},
               CMatView{Lt, q, 1, 0}, 0.0,
               MatView{N + (long)v.loff[t] * 2 * q, q, 1, 0});
        }
      }
      break;
    }
    case VSite::kCopy: {
      throw Error(kEinval, "absorb_right on a copy site");
    }
  }
}

DMps Engine::compress_chain(const std::vector<VSite>& ch_in, int cap, double tol,
                            Arena& out, hipStream_t s,
                            std::vector<double>* disc,
                            std::vector<std::vector<double>>* sigmas,
                            int centre) {
  const int n = (int)ch_in.size();
  MPSV_CHECK(n >= 2, kEinval, "compression needs at least two sites");
  MPSV_CHECK(centre >= 0 && centre < n, kEinval, "centre site out of range");
  MPSV_CHECK(centre == 0 || !sigmas, kEinval,
             "Schmidt values come from the plain sweep");
  cap = cap_or_inf(cap);
  const bool ig = p_.order == 4 && n == p_.n() && !sigmas;
  ArenaScope sc(work());
  // ---- right dense region.  Where the sites j..n-1 span no more indices
  // than the bond entering them (2^(n-j) <= r_(j-1)), that part of the
  // chain is contracted exactly into a dense block D (r_(j_R-1) x
  // 2^(n-j_R)); it is re-expressed as one dense core followed by
  // natural-basis copy cores.  The represented tensor, and therefore every
  // matricisation the truncation sweep sees, is unchanged.
  int jR = n;
  for (int j = n - 1; j >= 1; --j) {
    if (n - j > 30) break;
    if ((1L << (n - j)) <= (long)ch_in[j - 1].r) jR = j; else break;
  }
  std::vector<VSite> chv;
  const std::vector<VSite>* chp = &ch_in;
  if (jR <= n - 2) {
    double* Lb = work().alloc(1);
    fill(s, Lb, 1, 1.0);
    int q = 1;
    for (int j = n - 1; j >= jR; --j) {
      double* Nb = work().alloc((size_t)ch_in[j].l * 2 * q);
      absorb_right(ch_in[j], Lb, q, Nb, s);
      Lb = Nb;
      q *= 2;
    }
    chv.assign(ch_in.begin(), ch_in.begin() + jR);
    VSite d;
    d.kind = VSite::kDense;
    d.l = ch_in[jR].l;
    d.r = q / 2;
    d.A = Core{Lb, d.l, d.r};
    chv.push_back(d);
    for (int j = jR + 1; j < n; ++j) {
      VSite c;
      c.kind = VSite::kCopy;
      c.l = 1 << (n - j);
      c.r = 1 << (n - j - 1);
      chv.push_back(c);
    }
    chp = &chv;
  }
  const std::vector<VSite>& ch = *chp;
  struct Fac {
    bool ident = true;
    int rows = 0, cols = 0;
    QrFactor qf;
  };
  std::vector<Fac> fac(n);
  // ---- (i) QR sweep left to right.  A block with no more rows than
  // columns keeps Q = I (any orthogonal Q is a valid left-canonical gauge
  // and the identity is exact); taller blocks are Householder-factored.
  double* R = work().alloc(1);
  fill(s, R, 1, 1.0);
  int p = 1;
  for (int j = 0; j < n - 1; ++j) {
    const int rows = 2 * p, cols = ch[j].r;
    // a natural-basis site leaves R (p x 2r) as it is: no copy
    double* M = R;
    if (ch[j].kind != VSite::kCopy) {
      M = work().alloc((size_t)rows * cols);
      absorb_left(ch[j], R, p, M, s);
    }
    fac[j].rows = rows;
    fac[j].cols = cols;
    if (rows <= cols) {
      fac[j].ident = true;
      R = M;
      p = rows;
    } else {
      fac[j].ident = false;
      double* Rn = work().alloc((size_t)cols * cols);
      qr_factor(s, work(), M, rows, cols, cols, fac[j].qf,
                MatView{Rn, cols, 1, 0});
      R = Rn;
      p = cols;
    }
  }
  double* X = R;
  if (ch[n - 1].kind != VSite::kCopy) {
    X = work().alloc((size_t)p * 2);
    absorb_left(ch[n - 1], R, p, X, s);
  }
  // ---- (ii) truncated SVD sweep right to left.  Centre-first (SI,
  // Modified Compression Scheme; centre > 0): the sites right of the centre
  // are only brought to right-canonical form (untruncated SVDs), the centre
  // SVD truncates the cut between sites centre-1 and centre and its U S
  // moves left, so the rest of this sweep compresses the left half G = [s_r
  // g_r]; the right half H = S V^T ... is compressed by a left-to-right
  // sweep afterwards and S^-1 joins the centre site's left bond.
  DMps res(n);
  // discarded weights: n - 1 per instance (instance i's at i * (n - 1))
  const long dstride = n - 1;
  if (disc) disc->assign((size_t)(n - 1) * inst_count(), 0.0);
  if (sigmas) sigmas->assign(n - 1, {});
  double* sig_c = nullptr;  // centre singular values (device, descending)
  int m = p, Dr = 1;
  for (int j = n - 1; j >= 1; --j) {
    const int c = 2 * Dr;
    // exact (cap and tol off): right of the centre (centre-first), and the
    // bonds inside a fused x_k v_k pair of the IG ordering (its sites of
    // dimension 4 are held as two binary sites whose bond is never cut)
    const bool exact = (centre > 0 && j > centre) || (ig && (j & 1));
    const int capj = exact ? INT_MAX : cap;
    const double tolj = exact ? 0.0 : tol;
    Arena& dst = (centre > 0 && j >= centre) ? work() : out;
    const int Dmax = std::min(std::min(capj, m), c);
    double* Vt = dst.alloc((size_t)Dmax * c);
    double* US = work().alloc((size_t)m * Dmax);
    const bool want_sg = sigmas || (centre > 0 && j == centre);
    double* sg = want_sg ? work().alloc((size_t)std::min(m, c)) : nullptr;
    if (centre > 0 && j == centre) sig_c = sg;
    // the discarded weight goes straight to its place (a deferred call
    // writes it when the deferred section ends)
    double* dsc = disc ? &(*disc)[j - 1] : nullptr;
    int D;
    if (tolj <= 0.0 && !want_sg && std::min(m, c) <= capj) {
      // Nothing to truncate (every value is kept): only the right-canonical
      // gauge is needed, and an orthogonal factor gives it exactly.  A tall
      // block (m > c) keeps Vt = I and US = X; a wide one is factored as
      // X^T = Q R, so Vt = Q^T and US = R^T.  The represented tensor and
      // every later cut are the same as with the SVD.
      if (m > c) {
        D = c;
        identity(s, Vt, c);
        US = X;
      } else {
        D = m;
        QrFactor lq;
        qr_factor_view(s, work(), CMatView{X, 1, c, 0}, c, m, lq,
                       MatView{US, 1, m, 0});
        // Q^T = (Q [I; 0])^T, the identity read from the state's
        // persistent copy when it is large enough
        CMatView I{ident_, kIdent, 1, 0};
        if (m > kIdent) {
          double* Ib = work().alloc((size_t)m * m);
          identity(s, Ib, m);
          I = CMatView{Ib, m, 1, 0};
        }
        qr_apply_q_view(s, work(), lq, I, m, MatView{Vt, 1, c, 0}, m);
      }
      if (dsc)
        for (int i = 0; i < inst_count(); ++i) dsc[i * dstride] = 0.0;
    } else {
      D = svd_truncate(s, work(), X, m, c, c, capj, tolj, Vt, US, sg, dsc,
                       outcomes(s), dstride);
    }
    if (sigmas) {
      auto& h = (*sigmas)[j - 1];
      h.resize((size_t)std::min(m, c));
      d2h(s, h.data(), sg, h.size() * sizeof(double));
      MPSV_HIP(hipStreamSynchronize(s));
    }
    res[j] = Core{Vt, D, Dr};
    const Fac& f = fac[j - 1];
    if (f.ident) {
      X = US;  // (2 p_{j-2}) x D = p_{j-2} x (2D)
    } else {
      // US is f.cols x D: Y = Q [US; 0] (f.rows x D), the zero rows implied
      double* Y = work().alloc((size_t)f.rows * D);
      qr_apply_q_view(s, work(), f.qf, CMatView{US, D, 1, 0}, f.cols,
                      MatView{Y, D, 1, 0}, D);
      X = Y;
    }
    m = f.rows / 2;
    Dr = D;
  }
  // first core: X is 2 x Dr
  Core c0{out.alloc((size_t)2 * Dr), 1, Dr};
  copy_doubles(s, c0.p, X, 2L * Dr);
  res[0] = c0;
  if (centre > 0)
    compress_right_half(res, centre, sig_c, cap, tol, out, s, disc);
  return res;
}

// Right half of the centre-first scheme.  res[centre] = V_c^T and
// res[centre+1..n-1] are right-canonical (work arena); sc holds the centre
// values.  H = diag(sc) res[centre] res[centre+1] ... is swept left to
// right: the carried C (l x l_j) times core j, as (2 l) x r, is M = U S W^T
// truncated; core j <- U and C <- S W^T.  The SVD routine factors M^T, so
// M^T = (US') Vt' gives U = Vt'^T and S W^T = (US')^T.  Last, S^-1 is
// folded into the left bond of the centre core.
void Engine::compress_right_half(DMps& res, int centre, const double* sc,
                                 int cap, double tol, Arena& out, hipStream_t s,
                                 std::vector<double>* disc) {
  const int n = (int)res.size();
  const int Dc = res[centre].l;
  double* H = work().alloc((size_t)res[centre].size());
  scale_rows(s, res[centre].p, Dc, 2L * res[centre].r, sc, false, H);
  Core cur{H, Dc, res[centre].r};
  const double* C = nullptr;  // carry, (l x cur.l) read through view Cv
  CMatView Cv{nullptr, 0, 0, 0};
  int l = Dc;
  for (int j = centre; j < n - 1; ++j) {
    const int r = cur.r, rows = 2 * l;
    // Xt = M^T (r x rows): element (b, 2 i + t) = sum_a C[i][a] A[a][t][b]
    double* Xt = work().alloc((size_t)r * rows);
    if (C) {
      gemm(s, l, r, cur.l, 1.0, Cv, CMatView{cur.p, 2L * r, 1, r}, 0.0,
           MatView{Xt, 2, rows, 1}, 2);
    } else {
      copy_view(s, CMatView{cur.p, 2L * r, 1, 0}, l, MatView{Xt, 2, rows, 0}, l,
                r);
      copy_view(s, CMatView{cur.p + r, 2L * r, 1, 0}, l,
                MatView{Xt + 1, 2, rows, 0}, l, r);
    }
    const int Dmax = std::min(std::min(cap, r), rows);
    double* Vt = work().alloc((size_t)Dmax * rows);
    double* US = work().alloc((size_t)r * Dmax);
    const int D = svd_truncate(s, work(), Xt, r, rows, rows, cap, tol, Vt, US,
                               nullptr, disc ? &(*disc)[j] : nullptr,
                               outcomes(s), n - 1);
    // core j = Vt^T: (rows x D), row 2 i + t
    Core A{out.alloc((size_t)rows * D), l, D};
    copy_view(s, CMatView{Vt, 1, rows, 0}, rows, MatView{A.p, D, 1, 0}, rows, D);
    res[j] = A;
    C = US;
    Cv = CMatView{US, 1, D, 0};  // (US)^T, D x r
    l = D;
    cur = res[j + 1];
  }
  // last core: C (l x cur.l) times res[n-1] (cur.l x 2)
  Core last{out.alloc((size_t)l * 2), l, 1};
  if (C) {
    gemm(s, l, 2, cur.l, 1.0, Cv, CMatView{cur.p, 2, 1, 0}, 0.0,
         MatView{last.p, 2, 1, 0});
  } else {
    copy_doubles(s, last.p, cur.p, 2L * l);
  }
  res[n - 1] = last;
  // S^-1 into the centre core's left bond
  Core& A = res[centre];
  scale_rows(s, A.p, A.l, 2L * A.r, sc, true, A.p);
}

DMps Engine::compress_mps(const DMps& a, int cap, double tol, Arena& out,
                          hipStream_t s, std::vector<double>* disc,
                          int centre) {
  std::vector<VSite> ch(a.size());
  for (size_t j = 0; j < a.size(); ++j) {
    ch[j].kind = VSite::kDense;
    ch[j].A = a[j];
    ch[j].l = a[j].l;
    ch[j].r = a[j].r;
  }
  return compress_chain(ch, cap, tol, out, s, disc, nullptr,
                        centre < 0 ? centre_for((int)a.size()) : centre);
}

DMps Engine::apply_compress(const DMpo& W, const DMps& a, int cap, double tol,
                            Arena& out, hipStream_t s,
                            std::vector<double>* disc) {
  MPSV_CHECK(W.size() == a.size(), kEinval, "MPO/MPS length mismatch");
  std::vector<VSite> ch(a.size());
  for (size_t j = 0; j < a.size(); ++j) {
    ch[j].kind = VSite::kApply;
    ch[j].A = a[j];
    ch[j].W = W[j];
    ch[j].l = W[j].wl * a[j].l;
    ch[j].r = W[j].wr * a[j].r;
  }
  return compress_chain(ch, cap, tol, out, s, disc, nullptr,
                        centre_for((int)a.size()));
}

DMps Engine::add_terms(const std::vector<std::pair<double, const DMps*>>& terms,
                       int cap, Arena& out, hipStream_t s, double tol) {
  const int n = (int)terms[0].second->size();
  std::vector<VSite> ch(n);
  for (int j = 0; j < n; ++j) {
    VSite& v = ch[j];
    v.kind = VSite::kSum;
    v.pos = (j == 0) ? 0 : (j == n - 1 ? 2 : 1);
    int lo = 0, ro = 0;
    for (auto& t : terms) {
      const Core& A = (*t.second)[j];
      v.terms.push_back(A);
      v.coef.push_back(t.first);
      v.loff.push_back(lo);
      v.roff.push_back(ro);
      lo += A.l;
      ro += A.r;
    }
    v.l = (j == 0) ? 1 : lo;
    v.r = (j == n - 1) ? 1 : ro;
  }
  // disc_ keeps its storage (same length every time), so deferred
  // discarded weights can be written into it when the step's deferred
  // section ends
  return compress_chain(ch, cap, tol < 0 ? p_.tol : tol, out, s, &disc_,
                        nullptr, centre_for(n));
}

// The same tensor with the sites in reverse order: core (l, 2, r) ->
// (r, 2, l), last core first.
DMps Engine::reverse_mps(const DMps& a, Arena& ar, hipStream_t s) {
  const size_t L = a.size();
  DMps out(L);
  for (size_t j = 0; j < L; ++j) {
    const Core& A = a[L - 1 - j];
    out[j] = Core{ar.alloc(A.size()), A.r, A.l};
    reverse_core(s, A.p, A.l, A.r, out[j].p);
  }
  return out;
}

DMps Engine::copy_mps(const DMps& a, Arena& ar, hipStream_t s) {
  DMps out(a.size());
  for (size_t j = 0; j < a.size(); ++j) {
    out[j] = a[j];
    out[j].p = ar.alloc(a[j].size());
    copy_doubles(s, out[j].p, a[j].p, a[j].size());
  }
  return out;
}

// n(x) = dv * sum_j f(x, v_j): each v core summed over its bit (SI,
// Integration) and absorbed into the neighbouring x core.
DMps Engine::density(const DMps& g, Arena& ar, hipStream_t s, const DMps* wt) {
  const auto sites = site_list(p_.Lx, p_.Lv, p_.order);
  DMps xs;
  double* pend = nullptr;
  int pl = 0, pr = 0;
  for (size_t j = 0; j < sites.size(); ++j) {
    Core A = g[j];
    const bool vsite = sites[j].first == 1;
    double* Ms = nullptr;
    if (wt) {
      // the weight's bond joins f's (a-major): a v site is summed against
      // its weight core, an x site keeps its bit
      const Core& W = (*wt)[j];
      double* P = ar.alloc((size_t)A.l * W.l * (vsite ? 1 : 2) * A.r * W.r);
      pair_cores(s, A.p, A.l, A.r, W.p, W.l, W.r, vsite, P);
      A = Core{P, A.l * W.l, A.r * W.r};
      if (vsite) Ms = P;
    }
    if (vsite) {
      if (!Ms) {
        Ms = ar.alloc((size_t)A.l * A.r);
        sum_physical(s, A.p, A.l, A.r, Ms);
      }
      if (!xs.empty()) {
        Core& X = xs.back();
        double* Y = ar.alloc((size_t)X.l * 2 * A.r);
        gemm(s, X.l * 2, A.r, X.r, 1.0, CMatView{X.p, X.r, 1, 0},
             CMatView{Ms, A.r, 1, 0}, 0.0, MatView{Y, A.r, 1, 0});
        X.p = Y;
        X.r = A.r;
      } else if (pend == nullptr) {
        pend = Ms;
        pl = A.l;
        pr = A.r;
      } else {
        double* Y = ar.alloc((size_t)pl * A.r);
        gemm(s, pl, A.r, pr, 1.0, CMatView{pend, pr, 1, 0},
             CMatView{Ms, A.r, 1, 0}, 0.0, MatView{Y, A.r, 1, 0});
        pend = Y;
        pr = A.r;
      }
    } else {
      Core C = A;
      if (pend) {
        double* Y = ar.alloc((size_t)pl * 2 * A.r);
        gemm(s, pl, 2 * A.r, pr, 1.0, CMatView{pend, pr, 1, 0},
             CMatView{A.p, 2L * A.r, 1, 0}, 0.0, MatView{Y, 2L * A.r, 1, 0});
        C = Core{Y, pl, A.r};
        pend = nullptr;
      } else {
        double* Y = ar.alloc(A.size());
        copy_doubles(s, Y, A.p, A.size());
        C.p = Y;
      }
      xs.push_back(C);
    }
  }
  // x read fine to coarse (S2): back to the natural bit order
  if (p_.order == 2) xs = reverse_mps(xs, ar, s);
  // fold dv into the first core
  copy2d(s, 1, (int)xs[0].size(), p_.dv(), xs[0].p, xs[0].size(), xs[0].p,
         xs[0].size());
  return xs;
}

// E = compress(-G n, D_F, tol)  (Problem Statement eqs. 2-3)
DMps Engine::field(const DMps& g, Arena& ar, hipStream_t s) {
  // n lives below the compression's own workspace scope; E goes to `ar`
  ArenaScope sc(work());
  DMps n = density(g, work(), s);
  return apply_compress(gneg_, n, p_.df_max > 0 ? p_.df_max : INT_MAX, p_.tol,
                        ar, s);
}

// Full-chain MPO of diag(scale X) (x) vop (SI, Dot Product): the field term
// -(q/m) diag(E) (x) Dv, and the drift and temperature collision terms.
DMpo Engine::t2_mpo(const DMps& En, Arena& ar, hipStream_t s, double scale,
                    const DMpo& vop) {
  const auto sites = site_list(p_.Lx, p_.Lv, p_.order);
  // E (natural bit order) and Dv (held in chain order) as visited
  const DMps E = (p_.order == 2) ? reverse_mps(En, ar, s) : En;
  DMpo W(sites.size());
  int cx = 1, cv = 1, ix = 0, iv = 0;
  for (size_t j = 0; j < sites.size(); ++j) {
    MpoSite& m = W[j];
    if (sites[j].first == 0) {
      const Core& e = E[ix];
      double* Wd = ar.alloc((size_t)e.l * 4 * e.r);
      diag_mpo_site(s, e.p, e.l, e.r, ix == 0 ? scale : 1.0, Wd);
      ++ix;
      if (cv == 1) {
        m.W = Wd;
      } else {
        m.W = ar.alloc((size_t)e.l * cv * 4 * e.r * cv);
        kron_embed(s, Wd, e.l, 4, e.r, cv, 0, m.W);
      }
      m.wl = e.l * cv;
      m.wr = e.r * cv;
      cx = e.r;
    } else {
      const MpoSite& d = vop[iv++];
      if (cx == 1) {
        m.W = d.W;
      } else {
        m.W = ar.alloc((size_t)d.wl * cx * 4 * d.wr * cx);
        kron_embed(s, d.W, d.wl, 4, d.wr, cx, 1, m.W);
      }
      m.wl = d.wl * cx;
      m.wr = d.wr * cx;
      cv = d.wr;
    }
    m.Wmat = ar.alloc((size_t)m.wl * 4 * m.wr);
    mpo_left_matrix(s, m.W, m.wl, m.wr, m.Wmat);
  }
  return W;
}

// The collision terms with the drift v0(x) and the temperature vth^2(x) of
// g (Methods, Collision Operator): the moments <1,g>, <v,g>, <v^2/2,g> as
// x-MPS, on the x grid, divided there, back to x-MPS (compressed like the
// field), then -nu (diag(v0) (x) Dv) g and nu (diag(vth^2) (x) Dv Dv) g
// compressed at P5.
void Engine::moment_collision_terms(const DMps& g, Arena& out, hipStream_t s,
                                    DMps& Tu, DMps& Tt) {
  const long nx = p_.Nx();
  double* nd = out.alloc((size_t)nx);
  double* Pd = out.alloc((size_t)nx);
  double* Hd = out.alloc((size_t)nx);
  {
    ArenaScope sc(work());
    DMps n = density(g, work(), s);
    dense_of(n, nd, s);
    DMps P = density(g, work(), s, &vpoly_);
    dense_of(P, Pd, s);
    DMps H = density(g, work(), s, &v2poly_);
    dense_of(H, Hd, s);
  }
  double* v0 = out.alloc((size_t)nx);
  double* T = out.alloc((size_t)nx);
  dougherty_fields(s, nd, Pd, Hd, nx, v0, T);
  const double cut = p_.tol > 0 ? 1e-14 : 0.0;
  const int capf = p_.df_max > 0 ? p_.df_max : INT_MAX;
  DMps u = compress_mps(vector_mps(v0, p_.Lx, cut, out, s), capf, p_.tol, out, s);
  DMps t = compress_mps(vector_mps(T, p_.Lx, cut, out, s), capf, p_.tol, out, s);
  Tu = apply_compress(t2_mpo(u, out, s, -p_.nu, dv_), g, cap_for(5), p_.tol, out, s);
  Tt = apply_compress(t2_mpo(t, out, s, p_.nu, dv2_), g, cap_for(5), p_.tol, out, s);
}

// k = R(g) = -v d/dx g - (q/m) E d/dv g  (eq. 1, C = 0)
DMps Engine::rhs(const DMps& g, Arena& out, hipStream_t s, const DMps* Eext) {
  ArenaScope sc(tmp_);
  ArenaScope sc2(tmp2_);
  // The terms share only their input g.  T1 = -(Dx V) g (and the collision
  // term T3 = C g) are compressed on the side stream by a second host thread
  // (each factorisation of the sweep occupies one workgroup, so the sweeps
  // run side by side on the chip) while this thread computes the field and
  // compresses T2.
  MPSV_HIP(hipEventRecord(ev_fork_, s));
  MPSV_HIP(hipStreamWaitEvent(side_, ev_fork_, 0));
  DMps T1, T3;
  std::exception_ptr side_err;
  const Lanes lanes_here = lanes();
  auto side_lane = [&] {
    LanesScope ls(lanes_here);
    Arena* saved = tl_work;
    tl_work = &work2_;
    try {
      T1 = apply_compress(t1_, g, cap_for(5), p_.tol, tmp2_, side_);
      // the collision term also needs g alone: the side lane takes it too
      if (!coll_.empty()) T3 = apply_compress(coll_, g, cap_for(5), p_.tol, tmp2_, side_);
      MPSV_HIP(hipEventRecord(ev_join_, side_));
    } catch (...) {
      side_err = std::current_exception();
    }
    tl_work = saved;
  };
  // While a step graph is recorded, one host thread issues both lanes (the
  // side lane first): the recording gains nothing from a second thread,
  // and two threads must not add nodes to one capture at once.
  std::thread side;
  if (capturing_) {
    side_lane();
  } else {
    side = std::thread([&] {
      (void)hipSetDevice(device_);
      side_lane();
    });
  }
  auto join_side = [&] {
    if (side.joinable()) side.join();
  };
  DMps T2, T3u, T3t;
  try {
    DMps E;
    if (!Eext) E = field(g, tmp_, s);
    DMpo W2 = t2_mpo(Eext ? *Eext : E, tmp_, s, -p_.qm, dv_);
    T2 = apply_compress(W2, g, cap_for(5), p_.tol, tmp_, s);
    if (!dv2_.empty()) moment_collision_terms(g, tmp_, s, T3u, T3t);
  } catch (...) {
    join_side();
    if (!capturing_) (void)hipStreamSynchronize(side_);
    throw;
  }
  join_side();
  if (side_err) {
    if (!capturing_) (void)hipStreamSynchronize(side_);
    std::rethrow_exception(side_err);
  }
  MPSV_HIP(hipStreamWaitEvent(s, ev_join_, 0));
  if (coll_.empty()) return add_terms({{1.0, &T1}, {1.0, &T2}}, cap_for(4), out, s);
  if (dv2_.empty())
    return add_terms({{1.0, &T1}, {1.0, &T2}, {1.0, &T3}}, cap_for(4), out, s);
  return add_terms({{1.0, &T1}, {1.0, &T2}, {1.0, &T3}, {1.0, &T3u}, {1.0, &T3t}},
                   cap_for(4), out, s);
}

void Engine::commit(const DMps& fn, hipStream_t s) {
  // finiteness check first: the state only changes when the step is clean
  check_finite(fn, s);
  install(fn, s);
}

void Engine::check_finite(const DMps& fn, hipStream_t s) {
  fill_int(s, dflag_, 1, 0);
  for (auto& c : fn) count_nonfinite(s, c.p, c.size(), dflag_);
  // one flag per instance of the lanes
  const int ni = inst_count();
  int* bad = (int*)flags_host_.get((size_t)ni * sizeof(int));
  lanes_d2h(s, bad, dflag_, sizeof(int));
  MPSV_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < ni; ++i)
    if (bad[i])
      throw Error(kEnumeric, (ni > 1 ? "instance " + std::to_string(i) + ": " : std::string()) +
                                 "non-finite values in the new state");
}

void Engine::install(const DMps& fn, hipStream_t s) {
  state_.reset();
  f_ = copy_mps(fn, state_, s);
}

// Explicit direct sum of MPS of the same length (SI, Addition): block-
// diagonal cores, each term's scalar in its first core.
DMps Engine::direct_sum(const std::vector<std::pair<double, const DMps*>>& t,
                        Arena& ar, hipStream_t s) {
  const int n = (int)t[0].second->size();
  DMps out(n);
  for (int j = 0; j < n; ++j) {
    int L = 0, R = 0;
    for (auto& x : t) {
      L += (*x.second)[j].l;
      R += (*x.second)[j].r;
    }
    if (j == 0) L = 1;
    if (j == n - 1) R = 1;
    Core C{ar.alloc((size_t)L * 2 * R), L, R};
    fill(s, C.p, C.size(), 0.0);
    int lo = 0, ro = 0;
    for (auto& x : t) {
      const Core& A = (*x.second)[j];
      // A as (2 l) x r rows at row 2 lo, column ro of C as (2 L) x R
      copy2d(s, 2 * A.l, A.r, j == 0 ? x.first : 1.0, A.p, A.r,
             C.p + (long)2 * lo * R + ro, R);
      if (j > 0) lo += A.l;
      if (j < n - 1) ro += A.r;
    }
    out[j] = C;
  }
  return out;
}

// E of several species sharing x (Problem Statement eqs. 2-3 with the
// charge density of every species): rho = sum_s (-q_s) n_s formed exactly,
// E = compress(-G rho, D_F, tol) with the first species' settings.  The
// result and its inputs live in es[0]'s arena `ar`.
DMps field_of_species(const std::vector<Engine*>& es, const std::vector<double>& q,
                      const std::vector<const DMps*>& gs, Arena& ar, hipStream_t s) {
  Engine& e0 = *es[0];
  std::vector<DMps> ns(es.size());
  for (size_t i = 0; i < es.size(); ++i) ns[i] = es[i]->density(*gs[i], ar, s);
  std::vector<std::pair<double, const DMps*>> t;
  for (size_t i = 0; i < es.size(); ++i) t.push_back({-q[i], &ns[i]});
  const DMps rho = (es.size() == 1) ? ns[0] : e0.direct_sum(t, ar, s);
  if (es.size() == 1 && q[0] != -1.0) {
    // one species of another charge: scale its density instead
    copy2d(s, 1, (int)rho[0].size(), -q[0], rho[0].p, rho[0].size(), rho[0].p,
           rho[0].size());
  }
  return e0.apply_compress(e0.gneg_, rho, e0.p_.df_max > 0 ? e0.p_.df_max : INT_MAX,
                           e0.p_.tol, ar, s);
}

// One RK4 step of several species with a shared field (each stage's E from
// all of them), every species with its own compression points, committed
// for all or for none.
void step_species(const std::vector<Engine*>& es, const std::vector<double>& q,
                  hipStream_t s) {
  const size_t S = es.size();
  for (auto* e : es) MPSV_CHECK(!e->f_.empty(), kEinval, "state not initialised");
  Engine& e0 = *es[0];
  // the species share the reflector-application choice (checked at
  // creation); its lanes carry it to every launch of the step
  LanesScope ls(e0.one_lane(0));
  const double h = e0.p_.dt;
  for (auto* e : es) e->step_.reset();
  for (auto* e : es) {
    MPSV_CHECK(e->nin_ == 1, kEinval, "species are single instances");
    e->out_main_.begin();
    e->out_side_.begin();
  }
  std::vector<DMps> fn(S);
  try {
    auto R = [&](const std::vector<const DMps*>& gs) {
      DMps E = field_of_species(es, q, gs, e0.step_, s);
      std::vector<DMps> k(S);
      for (size_t i = 0; i < S; ++i) k[i] = es[i]->rhs(*gs[i], es[i]->step_, s, &E);
      return k;
    };
    auto stage = [&](const std::vector<DMps>& k, double c) {
      std::vector<DMps> g(S);
      for (size_t i = 0; i < S; ++i)
        g[i] = es[i]->add_terms({{1.0, &es[i]->f_}, {c, &k[i]}}, es[i]->cap_for(2),
                                es[i]->step_, s);
      return g;
    };
    auto ptrs = [](const std::vector<DMps>& v) {
      std::vector<const DMps*> p;
      for (auto& x : v) p.push_back(&x);
      return p;
    };
    std::vector<const DMps*> f0;
    for (auto* e : es) f0.push_back(&e->f_);
    const auto k1 = R(f0);
    const auto g2 = stage(k1, 0.5 * h);
    const auto k2 = R(ptrs(g2));
    const auto g3 = stage(k2, 0.5 * h);
    const auto k3 = R(ptrs(g3));
    const auto g4 = stage(k3, h);
    const auto k4 = R(ptrs(g4));
    for (size_t i = 0; i < S; ++i) {
      Engine& e = *es[i];
      DMps Sk = e.add_terms({{1.0, &k1[i]}, {2.0, &k2[i]}, {2.0, &k3[i]}, {1.0, &k4[i]}},
                            e.cap_for(3), e.step_, s);
      fn[i] = e.add_terms({{1.0, &e.f_}, {h / 6.0, &Sk}}, cap_or_inf(e.p_.chi_max),
                          e.step_, s);
    }
    for (auto* e : es) e->out_side_.end(e->side_);
    for (auto* e : es) e->out_main_.end(s);
  } catch (...) {
    for (auto* e : es) e->out_side_.cancel(e->side_);
    for (auto* e : es) e->out_main_.cancel(s);
    throw;
  }
  for (size_t i = 0; i < S; ++i) es[i]->check_finite(fn[i], s);
  for (size_t i = 0; i < S; ++i) {
    es[i]->install(fn[i], s);
    es[i]->t_ += h;
    ++es[i]->steps_;
  }
}

void field_species_dense(const std::vector<Engine*>& es, const std::vector<double>& q,
                         double* E_out, double* energy, hipStream_t s) {
  Engine& e0 = *es[0];
  ArenaScope sc(e0.tmp_);
  std::vector<const DMps*> gs;
  for (auto* e : es) gs.push_back(&e->f_);
  DMps E = field_of_species(es, q, gs, e0.tmp_, s);
  const long nx = e0.p_.Nx();
  double* Ed = E_out ? E_out : e0.tmp_.alloc((size_t)nx);
  e0.dense_of(E, Ed, s);
  if (energy) {
    double* w = e0.tmp_.alloc(1);
    sum_squares(s, Ed, nx, 0.5 * e0.p_.dx(), w);
    d2h(s, energy, w, sizeof(double));
  }
  MPSV_HIP(hipStreamSynchronize(s));
}

std::vector<double> Engine::entanglement(hipStream_t s, int inst) {
  MPSV_CHECK(!f_.empty(), kEinval, "state not initialised");
  check_instance(inst);
  LanesScope ls(one_lane(inst));
  ArenaScope sc(tmp_);
  std::vector<VSite> ch(f_.size());
  for (size_t j = 0; j < f_.size(); ++j) {
    ch[j].kind = VSite::kDense;
    ch[j].A = f_[j];
    ch[j].l = f_[j].l;
    ch[j].r = f_[j].r;
  }
  std::vector<std::vector<double>> sig;
  compress_chain(ch, INT_MAX, 0.0, tmp_, s, nullptr, &sig);
  std::vector<double> ee(sig.size(), 0.0);
  for (size_t b = 0; b < sig.size(); ++b) {
    double tot = 0.0;
    for (double x : sig[b]) tot += x * x;
    if (tot <= 0.0) continue;
    double e = 0.0;
    for (double x : sig[b]) {
      const double t = x * x / tot;
      if (t > 0.0) e -= t * std::log2(t);
    }
    ee[b] = e;
  }
  return ee;
}

double Engine::step_size(hipStream_t s) {
  if (p_.cfl <= 0) return p_.dt;
  LanesScope ls(one_lane(0));  // adaptive steps: one instance (checked at creation)
  // eq. CFL for one collisionless species, |E|_max of the current state
  ArenaScope sc(step_);
  DMps E = field(f_, step_, s);
  const long nx = p_.Nx();
  double* Ed = step_.alloc((size_t)nx);
  dense_of(E, Ed, s);
  std::vector<double> h((size_t)nx);
  d2h(s, h.data(), Ed, (size_t)nx * sizeof(double));
  MPSV_HIP(hipStreamSynchronize(s));
  double emax = 0.0;
  for (double e : h) emax = std::max(emax, std::fabs(e));
  MPSV_CHECK(std::isfinite(emax), kEnumeric, "non-finite field");
  const double vmax = std::max(std::fabs(p_.v_min), std::fabs(p_.v_max));
  double inv = vmax / p_.dx() + std::fabs(p_.qm) * emax / p_.dv();
  if (p_.nu != 0.0)
    inv += p_.nu * vmax / p_.dv() + 2.0 * p_.nu * p_.nu_vth * p_.nu_vth / (p_.dv() * p_.dv());
  return p_.cfl / inv;
}

void Engine::step(hipStream_t s) {
  MPSV_CHECK(!f_.empty(), kEinval, "state not initialised");
  step_.reset();
  const double h = step_size(s);
  step_.reset();
  // every instance of a batch in lock-step: each launch covers them all
  LanesScope ls(all_lanes());
  if (!graph_eligible()) {
    step_eager(h, s);
  } else {
    // On the instance's own stream, ordered after earlier work on s; later
    // work on s waits for the step.
    MPSV_HIP(hipEventRecord(ev_in_, s));
    MPSV_HIP(hipStreamWaitEvent(own_, ev_in_, 0));
    const std::vector<Core> key(f_.begin(), f_.end());
    if (gexec_ && same_cores(key, graph_key_)) {
      step_replay(own_);
    } else if (same_cores(key, warm_key_)) {
      step_capture(h, own_);
      graph_key_ = key;
    } else {
      // first step from this state layout: eager, which also sizes every
      // workspace the capture will use
      step_eager(h, own_);
      warm_key_ = key;
    }
    MPSV_HIP(hipEventRecord(ev_out_, own_));
    MPSV_HIP(hipStreamWaitEvent(s, ev_out_, 0));
  }
  t_ += h;
  ++steps_;
}

bool Engine::graph_eligible() const {
  static const bool env_off = [] {
    const char* e = std::getenv("MPSV_STEP_GRAPH");
    return e && std::atoi(e) == 0;
  }();
  // a replay needs the same shapes every step: fixed rank (tol = 0, every
  // SVD keeps min(cap, k)) and a fixed dt; timing probes need the launches
  return graph_on_ && !env_off && p_.tol <= 0.0 && p_.cfl <= 0.0 &&
         !prof_enabled();
}

bool Engine::same_cores(const std::vector<Core>& a, const std::vector<Core>& b) {
  if (a.size() != b.size()) return false;
  for (size_t j = 0; j < a.size(); ++j)
    if (a[j].p != b[j].p || a[j].l != b[j].l || a[j].r != b[j].r) return false;
  return true;
}

void Engine::step_eager(double h, hipStream_t s) {
  // Fixed-rank factorisations (tol = 0) report their outcome at the end of
  // the step instead of one host round trip each; a failure still fails
  // the step before anything is committed.
  out_main_.begin();
  out_side_.begin();
  try {
    step_stages(h, s);
    out_side_.end(side_);
    out_main_.end(s);
  } catch (...) {
    out_side_.cancel(side_);
    out_main_.cancel(s);
    throw;
  }
  commit(staged_, s);
  staged_.clear();
}

// Records the launches of one step (both streams, joined by the fork and
// join events of rhs) into a graph instead of running them, then replays
// it.  The graph holds the addresses of this state layout: the committed
// state, the arenas' workspace and the outcome slots, which stay put while
// the bonds do not change.
void Engine::step_capture(double h, hipStream_t s) {
  if (gexec_) {
    (void)hipGraphExecDestroy(gexec_);
    gexec_ = nullptr;
  }
  out_main_.begin();
  out_side_.begin();
  hipGraph_t g = nullptr;
  MPSV_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  capturing_ = true;
  try {
    step_stages(h, s);
  } catch (...) {
    capturing_ = false;
    (void)hipStreamEndCapture(s, &g);
    if (g) (void)hipGraphDestroy(g);
    (void)out_side_.take();
    (void)out_main_.take();
    throw;
  }
  capturing_ = false;
  MPSV_HIP(hipStreamEndCapture(s, &g));
  rec_own_ = out_main_.take();
  rec_side_ = out_side_.take();
  const hipError_t e = hipGraphInstantiate(&gexec_, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    gexec_ = nullptr;
    throw Error(kEdevice, std::string("graph instantiation: ") + hipGetErrorString(e));
  }
  graph_out_ = staged_;
  staged_.clear();
  ++graph_captures_;
  step_replay(s);
}

void Engine::step_replay(hipStream_t s) {
  out_main_.resume(rec_own_);
  out_side_.resume(rec_side_);
  try {
    MPSV_HIP(hipGraphLaunch(gexec_, s));
    out_main_.end(s);  // the whole graph, both lanes, has run
    out_side_.end(side_);
  } catch (...) {
    out_main_.cancel(s);
    out_side_.cancel(side_);
    throw;
  }
  commit(graph_out_, s);
  ++graph_replays_;
}

void Engine::step_stages(double h, hipStream_t s) {
  DMps k1 = rhs(f_, step_, s);
  DMps f2 = add_terms({{1.0, &f_}, {0.5 * h, &k1}}, cap_for(2), step_, s);
  DMps k2 = rhs(f2, step_, s);
  DMps f3 = add_terms({{1.0, &f_}, {0.5 * h, &k2}}, cap_for(2), step_, s);
  DMps k3 = rhs(f3, step_, s);
  DMps f4 = add_terms({{1.0, &f_}, {h, &k3}}, cap_for(2), step_, s);
  DMps k4 = rhs(f4, step_, s);
  DMps S = add_terms({{1.0, &k1}, {2.0, &k2}, {2.0, &k3}, {1.0, &k4}},
                     cap_for(3), step_, s);
  staged_ = add_terms({{1.0, &f_}, {h / 6.0, &S}}, cap_or_inf(p_.chi_max),
                      step_, s);
}

// ---------------------------------------------------------------- state io

// f0 = sum_r ax[r] (x) bv[r] as an MPS in the step arena (one instance):
// each 1-D profile by iterated SVD (eq. 4), then the separable terms
// merged in chain order and compressed to (chi, tol).
// Iterated SVD (eq. 4) run from the right end: X = u as 2^(L-1) x 2, SVD,
// keep V^T as the last core, carry U S; values below `cut` of the norm
// (relative discarded weight) are dropped, none with cut = 0.  Cores in ar,
// temporaries in the compression workspace.
DMps Engine::vector_mps(const double* u, int L, double cut, Arena& ar, hipStream_t s) {
  DMps m(L);
  ArenaScope sc(work());
  double* X = work().alloc((size_t)1 << L);
  copy_doubles(s, X, u, 1L << L);
  int rows = 1 << (L - 1), Dr = 1;
  for (int j = L - 1; j >= 1; --j) {
    const int c = 2 * Dr;
    const int Dmax = std::min(rows, c);
    double* Vt = ar.alloc((size_t)Dmax * c);
    double* US = work().alloc((size_t)rows * Dmax);
    const int D = svd_truncate(s, work(), X, rows, c, c, INT_MAX, cut, Vt, US,
                               nullptr, nullptr, outcomes(s), 0);
    m[j] = Core{Vt, D, Dr};
    X = US;
    rows /= 2;
    Dr = D;
  }
  Core c0{ar.alloc((size_t)2 * Dr), 1, Dr};
  copy_doubles(s, c0.p, X, 2L * Dr);
  m[0] = c0;
  return m;
}

DMps Engine::initial_state(int rank, const double* ax, const double* bv,
                           hipStream_t s) {
  MPSV_CHECK(rank >= 1, kEinval, "profile rank must be >= 1");
  MPSV_CHECK(inst_count() == 1, kEinval, "one instance at a time");
  // the caller's profiles enter the instance's workspace first (the
  // kernels below address instance-local buffers only)
  const long nx = (long)rank * p_.Nx(), nv = (long)rank * p_.Nv();
  double* axl = step_.alloc((size_t)nx);
  double* bvl = step_.alloc((size_t)nv);
  d2d_in(s, axl, ax, (size_t)nx * sizeof(double));
  d2d_in(s, bvl, bv, (size_t)nv * sizeof(double));
  // non-finite profiles are rejected
  fill_int(s, dflag_, 1, 0);
  count_nonfinite(s, axl, nx, dflag_);
  count_nonfinite(s, bvl, nv, dflag_);
  int bad = 0;
  d2h(s, &bad, dflag_, sizeof(int));
  MPSV_HIP(hipStreamSynchronize(s));
  MPSV_CHECK(bad == 0, kEinval, "non-finite values in the initial profiles");

  // 1-D vector -> MPS by iterated SVD (eq. 4).  The relative floor 1e-14
  // drops only numerically zero directions (a smooth profile keeps a
  // handful), whatever the problem's tolerance.
  auto tt = [&](const double* u, int L) { return vector_mps(u, L, 1e-14, step_, s); };
  std::vector<DMps> terms;
  {
    ArenaScope sc(work());
    for (int r = 0; r < rank; ++r) {
      DMps mx = tt(axl + (long)r * p_.Nx(), p_.Lx);
      DMps mv = tt(bvl + (long)r * p_.Nv(), p_.Lv);
      DMps full;
      if (p_.order != 1 && p_.order != 4) {
        // sequential: a dimension read fine to coarse enters reversed
        full = (p_.order == 2) ? reverse_mps(mx, step_, s) : mx;
        const DMps v = (p_.order == 3) ? reverse_mps(mv, step_, s) : mv;
        full.insert(full.end(), v.begin(), v.end());
      } else {
        int cx = 1, cv = 1;
        for (int k = 0; k < p_.Lx; ++k) {
          const Core& X = mx[k];
          Core cxk{step_.alloc((size_t)X.l * cv * 2 * X.r * cv), X.l * cv,
                   X.r * cv};
          kron_embed(s, X.p, X.l, 2, X.r, cv, 0, cxk.p);
          full.push_back(cxk);
          cx = X.r;
          const Core& V = mv[k];
          Core cvk{step_.alloc((size_t)V.l * cx * 2 * V.r * cx), V.l * cx,
                   V.r * cx};
          kron_embed(s, V.p, V.l, 2, V.r, cx, 1, cvk.p);
          full.push_back(cvk);
          cv = V.r;
        }
      }
      terms.push_back(full);
    }
  }
  std::vector<std::pair<double, const DMps*>> tl;
  for (auto& t : terms) tl.push_back({1.0, &t});
  if (rank == 1) return compress_mps(terms[0], cap_or_inf(p_.chi_max), p_.tol, step_, s);
  return add_terms(tl, cap_or_inf(p_.chi_max), step_, s);
}

void Engine::init_from_profiles(int rank, const double* ax, const double* bv,
                                hipStream_t s, int inst) {
  check_instance(inst);
  MPSV_CHECK(nin_ == 1, kEinval, "a batch is initialised by init_batch");
  LanesScope ls(one_lane(0));
  step_.reset();
  DMps f0 = initial_state(rank, ax, bv, s);
  commit(f0, s);
  t_ = 0.0;
  steps_ = 0;
}

// Every instance's own initial state, then all of them committed at once:
// they must come out with the same bond dimensions (profiles of the same
// kind; with tol = 0 only numerically zero directions are dropped).
void Engine::init_batch(const std::vector<int>& ranks,
                        const std::vector<const double*>& ax,
                        const std::vector<const double*>& bv, hipStream_t s) {
  MPSV_CHECK((int)ranks.size() == nin_ && (int)ax.size() == nin_ &&
                 (int)bv.size() == nin_,
             kEinval, "one profile pair per instance expected");
  std::vector<int> b0;
  std::vector<std::vector<double>> host((size_t)nin_);
  for (int i = 0; i < nin_; ++i) {
    LanesScope ls(one_lane(i));
    step_.reset();
    DMps f0 = initial_state(ranks[i], ax[i], bv[i], s);
    std::vector<int> b(f0.size() + 1, 1);
    long tot = 0;
    for (size_t j = 0; j < f0.size(); ++j) {
      b[j + 1] = f0[j].r;
      tot += f0[j].size();
    }
    b[0] = f0[0].l;
    if (i == 0) b0 = b;
    MPSV_CHECK(b == b0, kEinval,
               "instance " + std::to_string(i) +
                   ": its initial state has other bond dimensions than instance 0's");
    host[i].resize((size_t)tot);
    long off = 0;
    for (auto& c : f0) {
      d2h(s, host[i].data() + off, c.p, c.size() * sizeof(double));
      off += c.size();
    }
    MPSV_HIP(hipStreamSynchronize(s));
  }
  set_states_host(b0, host, s);
  t_ = 0.0;
  steps_ = 0;
}

// Cores of every instance (same bonds; host arrays, packed core by core)
// staged in the step arena at common addresses, then committed together.
void Engine::set_states_host(const std::vector<int>& bonds,
                             const std::vector<std::vector<double>>& packed,
                             hipStream_t s) {
  LanesScope ls(all_lanes());
  step_.reset();
  DMps a(n());
  for (int j = 0; j < n(); ++j) {
    a[j] = Core{nullptr, bonds[j], bonds[j + 1]};
    a[j].p = step_.alloc(a[j].size());
  }
  for (int i = 0; i < nin_; ++i) {
    long off = 0;
    for (auto& c : a) {
      MPSV_HIP(hipMemcpyAsync(shifted(c.p, (long)i * (long)chunk_), packed[i].data() + off,
                              c.size() * sizeof(double), hipMemcpyHostToDevice, s));
      off += c.size();
    }
  }
  commit(a, s);
}

static std::vector<Core> view_packed(const std::vector<int>& bonds, const double* packed,
                                     int n) {
  MPSV_CHECK((int)bonds.size() == n + 1 && bonds[0] == 1 && bonds[n] == 1, kEinval,
             "bond dimensions must have n+1 entries with unit ends");
  std::vector<Core> a((size_t)n);
  long off = 0;
  for (int j = 0; j < n; ++j) {
    MPSV_CHECK(bonds[j + 1] >= 1, kEinval, "bond dimension must be >= 1");
    a[j] = Core{const_cast<double*>(packed) + off, bonds[j], bonds[j + 1]};
    off += a[j].size();
  }
  return a;
}

// Packed device cores of every instance (same bonds) staged in the step
// arena at common addresses.
DMps Engine::stage_packed(const std::vector<int>& bonds,
                          const std::vector<const double*>& packed, hipStream_t s) {
  MPSV_CHECK((int)packed.size() == nin_, kEinval, "one set of cores per instance expected");
  const DMps v = view_packed(bonds, packed[0], n());
  DMps a(n());
  for (int j = 0; j < n(); ++j) {
    a[j] = v[j];
    a[j].p = step_.alloc(v[j].size());
  }
  for (int i = 0; i < nin_; ++i) {
    LanesScope ls(one_lane(i));
    const DMps vi = view_packed(bonds, packed[i], n());
    for (int j = 0; j < n(); ++j) d2d_in(s, a[j].p, vi[j].p, vi[j].size() * sizeof(double));
  }
  return a;
}

void Engine::set_state(const std::vector<int>& bonds, const double* packed,
                       hipStream_t s, int inst) {
  check_instance(inst);
  MPSV_CHECK(nin_ == 1, kEinval, "a batch takes its cores by set_states");
  set_states(bonds, {packed}, s);
}

void Engine::set_states(const std::vector<int>& bonds,
                        const std::vector<const double*>& packed, hipStream_t s) {
  LanesScope ls(all_lanes());
  step_.reset();
  DMps a = stage_packed(bonds, packed, s);
  commit(a, s);
}

void Engine::get_state(std::vector<int>& bonds, double* packed, hipStream_t s,
                       int inst) const {
  check_instance(inst);
  LanesScope ls(one_lane(inst));
  bonds = this->bonds();
  long off = 0;
  for (auto& c : f_) {
    if (packed) d2d_out(s, packed + off, c.p, c.size() * sizeof(double));
    off += c.size();
  }
}

void Engine::add_scaled(double alpha, const std::vector<int>& bonds,
                        const double* packed, hipStream_t s, int inst) {
  check_instance(inst);
  MPSV_CHECK(nin_ == 1, kEinval, "a batch adds by add_scaled_all");
  add_scaled_all({alpha}, bonds, {packed}, s);
}

// f_i <- compress(f_i + alpha_i g_i) for every instance (one set of bonds
// for all g_i).  One instance keeps the scalar in the sum's coefficient; a
// batch scales each g_i's first core by its alpha_i instead (the sum's
// coefficients are common to all instances).
void Engine::add_scaled_all(const std::vector<double>& alpha,
                            const std::vector<int>& bonds,
                            const std::vector<const double*>& packed, hipStream_t s) {
  MPSV_CHECK((int)alpha.size() == nin_, kEinval, "one scalar per instance expected");
  for (double a : alpha) MPSV_CHECK(std::isfinite(a), kEinval, "alpha must be finite");
  LanesScope ls(all_lanes());
  step_.reset();
  DMps g = stage_packed(bonds, packed, s);
  double coef = alpha[0];
  if (nin_ > 1) {
    coef = 1.0;
    for (int i = 0; i < nin_; ++i) {
      LanesScope l1(one_lane(i));
      copy2d(s, 1, (int)g[0].size(), alpha[i], g[0].p, g[0].size(), g[0].p, g[0].size());
    }
  }
  // a batch's truncations (tol = 0) report their outcomes at the end
  DMps fn;
  out_main_.begin();
  try {
    fn = add_terms({{1.0, &f_}, {coef, &g}}, cap_or_inf(p_.chi_max), step_, s);
    out_main_.end(s);
  } catch (...) {
    out_main_.cancel(s);
    throw;
  }
  commit(fn, s);
}

void Engine::dense_of(const DMps& a, double* out, hipStream_t s) {
  const int n = (int)a.size();
  ArenaScope sc(tmp_);
  long maxsz = 2L * a[0].r;
  long rows = 2;
  for (int j = 1; j < n; ++j) {
    rows *= 2;
    maxsz = std::max(maxsz, rows * (long)a[j].r);
  }
  double* b0 = tmp_.alloc(maxsz);
  double* b1 = tmp_.alloc(maxsz);
  copy_doubles(s, b0, a[0].p, a[0].size());
  long r = 2;  // rows of the current block
  double* cur = b0;
  double* nxt = b1;
  for (int j = 1; j < n; ++j) {
    double* dst = (j == n - 1) ? out : nxt;
    gemm(s, (int)r, 2 * a[j].r, a[j].l, 1.0, CMatView{cur, a[j].l, 1, 0},
         CMatView{a[j].p, 2L * a[j].r, 1, 0}, 0.0,
         MatView{dst, 2L * a[j].r, 1, 0});
    r *= 2;
    std::swap(cur, nxt);
  }
}

void Engine::to_dense(double* out_caller, hipStream_t s, int inst) {
  MPSV_CHECK(!f_.empty(), kEinval, "state not initialised");
  check_instance(inst);
  LanesScope ls(one_lane(inst));
  double* out = foreign(out_caller);
  if (p_.order == 0) {
    dense_of(f_, out, s);
  } else {
    ArenaScope sc(tmp_);
    double* v = tmp_.alloc((size_t)1 << n());
    dense_of(f_, v, s);
    if (p_.order == 1 || p_.order == 4)
      deinterleave(s, v, p_.Lx, out);
    else
      chain_to_grid(s, v, p_.Lx, p_.Lv, p_.order == 2, p_.order == 3, out);
  }
}

double Engine::full_contract(const DMps& g, const DMps& f, hipStream_t s) {
  ArenaScope sc(tmp_);
  double* E = tmp_.alloc(1);
  fill(s, E, 1, 1.0);
  int ga = 1, fa = 1;
  for (size_t j = 0; j < f.size(); ++j) {
    const Core& G = g[j];
    const Core& F = f[j];
    double* T = tmp_.alloc((size_t)ga * 2 * F.r);
    gemm(s, ga, 2 * F.r, fa, 1.0, CMatView{E, fa, 1, 0},
         CMatView{F.p, 2L * F.r, 1, 0}, 0.0, MatView{T, 2L * F.r, 1, 0});
    double* En = tmp_.alloc((size_t)G.r * F.r);
    for (int sidx = 0; sidx < 2; ++sidx)
      gemm(s, G.r, F.r, ga, 1.0, CMatView{G.p + sidx * G.r, 1, 2L * G.r, 0},
           CMatView{T + sidx * F.r, 2L * F.r, 1, 0}, sidx ? 1.0 : 0.0,
           MatView{En, F.r, 1, 0});
    E = En;
    ga = G.r;
    fa = F.r;
  }
  double h = 0.0;
  d2h(s, &h, E, sizeof(double));
  MPSV_HIP(hipStreamSynchronize(s));
  return h;
}

void Engine::density_field(double* n_out, double* E_out, hipStream_t s, int inst) {
  MPSV_CHECK(!f_.empty(), kEinval, "state not initialised");
  check_instance(inst);
  LanesScope ls(one_lane(inst));
  ArenaScope sc(step_);
  DMps nm = density(f_, step_, s);
  DMps E = field(f_, step_, s);
  if (n_out) dense_of(nm, foreign(n_out), s);
  if (E_out) dense_of(E, foreign(E_out), s);
  MPSV_HIP(hipStreamSynchronize(s));
}

void Engine::moments(double* n_out, double* E_out, double* scalars,
                     hipStream_t s, int inst) {
  MPSV_CHECK(!f_.empty(), kEinval, "state not initialised");
  check_instance(inst);
  LanesScope ls(one_lane(inst));
  ArenaScope sc(step_);
  DMps nm = density(f_, step_, s);
  DMps E = field(f_, step_, s);
  if (n_out) dense_of(nm, foreign(n_out), s);
  double* Ed = nullptr;
  if (E_out) {
    Ed = foreign(E_out);
    dense_of(E, Ed, s);
  }
  if (scalars) {
    ArenaScope sc2(tmp_);
    if (!Ed) {
      Ed = step_.alloc((size_t)p_.Nx());
      dense_of(E, Ed, s);
    }
    double* we = tmp_.alloc(1);
    sum_squares(s, Ed, p_.Nx(), 0.5 * p_.dx(), we);
    double hwe = 0.0;
    d2h(s, &hwe, we, sizeof(double));
    MPSV_HIP(hipStreamSynchronize(s));
    // mass = dx * sum_i n_i = dx dv <1, f>; momentum / kinetic with v, v^2/2
    double mass = 0.0;
    {
      // <1, n> over the x sites
      ArenaScope sc3(tmp_);
      DMps onesx(nm.size());
      for (size_t j = 0; j < nm.size(); ++j) {
        onesx[j] = Core{tmp_.alloc(2), 1, 1};
        fill(s, onesx[j].p, 2, 1.0);
      }
      mass = p_.dx() * full_contract(onesx, nm, s);
    }
    const double w = p_.dx() * p_.dv();
    scalars[0] = mass;
    scalars[1] = w * full_contract(vpoly_, f_, s);
    scalars[2] = w * full_contract(v2poly_, f_, s);
    scalars[3] = hwe;
  }
  MPSV_HIP(hipStreamSynchronize(s));
}

}  // namespace mpsv
