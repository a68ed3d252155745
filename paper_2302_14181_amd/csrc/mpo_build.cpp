// Host construction of the order-N MPO approximation of exp(tau H).
//
// The Hamiltonian is a first-degree MPO in Jordan form (Sec. 2.3): level 1 (nothing has acted),
// level 2 (acting, dimension chi), level 3 (done); H[1,1] = H[3,3] = I, H[1,2] = C,
// H[1,3] = Dloc, H[2,2] = A, H[2,3] = B.  Powers H^N live on level tuples t in {1,2,3}^N whose
// virtual dimension is chi^(number of 2s) (Sec. 2.5).  The construction:
//   V1: H^N -> fold of the {1,3}-only levels into (1,...,1) (Alg. 1, Sec. 3)
//           -> merge of equivalent levels (Alg. 2, Sec. 4)
//   V2: H^N -> extension by the order-(N+1) terms that overlap at most N times (Alg. 3, Sec. 5)
//           -> Alg. 1 -> Alg. 2 -> approximate compression of the 1-free levels (Alg. 4, Sec. 6)
// Readings where the printed pseudocode is ambiguous (same as the documented design notes):
//   Alg. 3 visits target levels without any 1; Alg. 2 moves 3s to the back for column merges;
//   Alg. 4 visits 1-free levels with at least one 3 and folds them into the level whose 3s are
//   turned into 1s, written with the 1s in front; all loops visit levels in lexicographic order.
//
// Levels are stored as base-3 codes, position 0 most significant, digit = value - 1, so numeric
// order is lexicographic order. A block between two levels is a dense tensor
// [v_row][d][d][v_col] of complex doubles.

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstddef>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"

namespace mpoevo {
namespace {

using cplx = std::complex<double>;

struct Tensor4 {  // [vr][d][d][vc]
  int vr = 0, vc = 0, d = 0;
  std::vector<cplx> a;
  Tensor4() = default;
  Tensor4(int vr_, int d_, int vc_) : vr(vr_), vc(vc_), d(d_), a((size_t)vr_ * d_ * d_ * vc_) {}
  cplx& at(int r, int so, int si, int c) { return a[(((size_t)r * d + so) * d + si) * vc + c]; }
  const cplx& at(int r, int so, int si, int c) const { return a[(((size_t)r * d + so) * d + si) * vc + c]; }
};

struct Level {
  std::vector<int> t;  // values 1..3
  int code() const {
    int c = 0;
    for (int x : t) c = c * 3 + (x - 1);
    return c;
  }
  int count(int v) const { return (int)std::count(t.begin(), t.end(), v); }
};

Level decode(int code, int N) {
  Level l;
  l.t.assign(N, 1);
  for (int j = N - 1; j >= 0; --j) {
    l.t[j] = code % 3 + 1;
    code /= 3;
  }
  return l;
}

int ipow(int b, int e) {
  int r = 1;
  while (e-- > 0) r *= b;
  return r;
}

double factorial(int n) {
  double f = 1;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

struct Jordan {
  int d, chi;
  const double *A, *B, *C, *D;
  cplx get(const double* p, size_t idx) const { return cplx(p[2 * idx], p[2 * idx + 1]); }
  // block of a single copy between levels x -> y; returns false if structurally zero
  bool single(int x, int y, Tensor4& out) const {
    if ((x == 1 && y == 1) || (x == 3 && y == 3)) {
      out = Tensor4(1, d, 1);
      for (int s = 0; s < d; ++s) out.at(0, s, s, 0) = 1.0;
      return true;
    }
    if (x == 1 && y == 2) {
      out = Tensor4(1, d, chi);
      for (int k = 0; k < chi; ++k)
        for (int so = 0; so < d; ++so)
          for (int si = 0; si < d; ++si) out.at(0, so, si, k) = get(C, ((size_t)k * d + so) * d + si);
      return true;
    }
    if (x == 1 && y == 3) {
      out = Tensor4(1, d, 1);
      for (int so = 0; so < d; ++so)
        for (int si = 0; si < d; ++si) out.at(0, so, si, 0) = get(D, (size_t)so * d + si);
      return true;
    }
    if (x == 2 && y == 2) {
      out = Tensor4(chi, d, chi);
      for (int k = 0; k < chi; ++k)
        for (int l = 0; l < chi; ++l)
          for (int so = 0; so < d; ++so)
            for (int si = 0; si < d; ++si)
              out.at(k, so, si, l) = get(A, (((size_t)k * chi + l) * d + so) * d + si);
      return true;
    }
    if (x == 2 && y == 3) {
      out = Tensor4(chi, d, 1);
      for (int k = 0; k < chi; ++k)
        for (int so = 0; so < d; ++so)
          for (int si = 0; si < d; ++si) out.at(k, so, si, 0) = get(B, ((size_t)k * d + so) * d + si);
      return true;
    }
    return false;
  }
  // block of H^n between level tuples a and b (copy 1 acts leftmost on the physical legs,
  // virtual indices are Kronecker products in position order)
  bool power(const std::vector<int>& a, const std::vector<int>& b, Tensor4& out) const {
    Tensor4 acc;
    bool first = true;
    for (size_t j = 0; j < a.size(); ++j) {
      Tensor4 f;
      if (!single(a[j], b[j], f)) return false;
      if (first) {
        acc = std::move(f);
        first = false;
        continue;
      }
      Tensor4 nxt(acc.vr * f.vr, d, acc.vc * f.vc);
      for (int r1 = 0; r1 < acc.vr; ++r1)
        for (int r2 = 0; r2 < f.vr; ++r2)
          for (int c1 = 0; c1 < acc.vc; ++c1)
            for (int c2 = 0; c2 < f.vc; ++c2)
              for (int so = 0; so < d; ++so)
                for (int si = 0; si < d; ++si) {
                  cplx s = 0;
                  for (int x = 0; x < d; ++x) s += acc.at(r1, so, x, c1) * f.at(r2, x, si, c2);
                  nxt.at(r1 * f.vr + r2, so, si, c1 * f.vc + c2) = s;
                }
      acc = std::move(nxt);
    }
    out = std::move(acc);
    return true;
  }
};

// Operator-valued level matrix: present levels (codes) and nonzero blocks.
struct LevelMat {
  int N;
  std::set<int> present;
  std::map<std::pair<int, int>, Tensor4> blk;

  void accumulate(int r, int c, const Tensor4& t, cplx w) {
    auto key = std::make_pair(r, c);
    auto it = blk.find(key);
    if (it == blk.end()) {
      Tensor4 s = t;
      for (auto& x : s.a) x *= w;
      blk.emplace(key, std::move(s));
    } else {
      for (size_t i = 0; i < t.a.size(); ++i) it->second.a[i] += w * t.a[i];
    }
  }
  void drop(int c) {
    present.erase(c);
    for (auto it = blk.begin(); it != blk.end();) {
      if (it->first.first == c || it->first.second == c) it = blk.erase(it);
      else ++it;
    }
  }
  // add column src (times w) into column dst, for every present row
  void add_column(int src, int dst, cplx w) {
    std::vector<std::pair<int, Tensor4>> adds;
    for (int r : present) {
      auto it = blk.find({r, src});
      if (it != blk.end()) adds.emplace_back(r, it->second);
    }
    for (auto& p : adds) accumulate(p.first, dst, p.second, w);
  }
  void add_row(int src, int dst) {
    std::vector<std::pair<int, Tensor4>> adds;
    for (int c : present) {
      auto it = blk.find({src, c});
      if (it != blk.end()) adds.emplace_back(c, it->second);
    }
    for (auto& p : adds) accumulate(dst, p.first, p.second, 1.0);
  }
};

std::vector<int> stable_front(const std::vector<int>& t, int v) {  // entries equal to v first
  std::vector<int> o;
  for (int x : t) if (x == v) o.push_back(x);
  for (int x : t) if (x != v) o.push_back(x);
  return o;
}
std::vector<int> stable_back(const std::vector<int>& t, int v) {  // entries equal to v last
  std::vector<int> o;
  for (int x : t) if (x != v) o.push_back(x);
  for (int x : t) if (x == v) o.push_back(x);
  return o;
}
int code_of(const std::vector<int>& t) {
  Level l;
  l.t = t;
  return l.code();
}

LevelMat power_matrix(const Jordan& H, int N) {
  LevelMat M;
  M.N = N;
  const int nl = ipow(3, N);
  for (int c = 0; c < nl; ++c) M.present.insert(c);
  for (int r = 0; r < nl; ++r) {
    Level a = decode(r, N);
    for (int c = 0; c < nl; ++c) {
      Level b = decode(c, N);
      bool ok = true;
      for (int j = 0; j < N; ++j) ok = ok && (a.t[j] <= b.t[j]);
      if (!ok) continue;
      Tensor4 t;
      if (H.power(a.t, b.t, t)) M.blk.emplace(std::make_pair(r, c), std::move(t));
    }
  }
  return M;
}

// Alg. 3 on the raw H^N (see the file comment for the reading of its conditions).
void extension(LevelMat& M, const Jordan& H, cplx tau) {
  const int N = M.N;
  const double base = factorial(N) / factorial(N + 1);
  std::vector<std::pair<std::pair<int, int>, Tensor4>> adds;
  for (int r : M.present) {
    Level a = decode(r, N);
    if (a.count(2) == 0 && a.count(3) > 0) continue;
    for (int c : M.present) {
      Level b = decode(c, N);
      if (b.count(1) > 0) continue;
      Tensor4 acc;
      bool have = false;
      for (int pos_a = 0; pos_a <= N; ++pos_a) {
        std::vector<int> ae = a.t;
        ae.insert(ae.begin() + pos_a, 1);
        const int n1 = (int)std::count(ae.begin(), ae.end(), 1);
        for (int pos_b = 0; pos_b <= N; ++pos_b) {
          std::vector<int> be = b.t;
          be.insert(be.begin() + pos_b, 3);
          const int n3 = (int)std::count(be.begin(), be.end(), 3);
          Tensor4 t;
          if (!H.power(ae, be, t)) continue;
          const cplx w = tau * base / double(n1 * n3);
          if (!have) {
            acc = t;
            for (auto& x : acc.a) x *= w;
            have = true;
          } else {
            for (size_t i = 0; i < t.a.size(); ++i) acc.a[i] += w * t.a[i];
          }
        }
      }
      if (have) adds.emplace_back(std::make_pair(r, c), std::move(acc));
    }
  }
  for (auto& p : adds) M.accumulate(p.first.first, p.first.second, p.second, 1.0);
}

// Alg. 1: fold the levels made of 1s and k 3s (k = 1..N) into (1,...,1).
void fold(LevelMat& M, cplx tau) {
  const int N = M.N;
  const int one = 0;  // code of (1,...,1)
  for (int k = 1; k <= N; ++k) {
    const cplx w = std::pow(tau, k) * (factorial(N - k) / factorial(N));
    std::vector<int> targets;
    for (int c : M.present) {
      Level l = decode(c, N);
      if (l.count(2) == 0 && l.count(3) == k) targets.push_back(c);
    }
    for (int c : targets) {
      M.add_column(c, one, w);
      M.drop(c);
    }
  }
}

// Alg. 2: merge levels with equal left environments (rows) or equal right environments (columns).
void exact_compress(LevelMat& M) {
  const int N = M.N;
  std::vector<int> order(M.present.begin(), M.present.end());
  for (int c : order) {
    if (!M.present.count(c)) continue;
    Level l = decode(c, N);
    const int n1 = l.count(1), n3 = l.count(3);
    if (n3 <= n1) {
      const int s = code_of(stable_front(l.t, 1));
      if (s != c) {
        M.add_row(c, s);
        M.drop(c);
      }
    } else {
      const int s = code_of(stable_back(l.t, 3));
      if (s != c) {
        M.add_column(c, s, 1.0);
        M.drop(c);
      }
    }
  }
}

// Alg. 4: fold every 1-free level with k >= 1 threes into its 3->1 counterpart.
bool approx_compress(LevelMat& M, cplx tau, std::string& err) {
  const int N = M.N;
  std::vector<int> order(M.present.begin(), M.present.end());
  for (int c : order) {
    if (!M.present.count(c)) continue;
    Level l = decode(c, N);
    if (l.count(1) > 0 || l.count(3) == 0) continue;
    const int k = l.count(3);
    std::vector<int> t = l.t;
    for (int& x : t) if (x == 3) x = 1;
    const int target = code_of(stable_front(t, 1));
    if (!M.present.count(target)) {
      err = "approximate compression: target level missing";
      return false;
    }
    M.add_column(c, target, std::pow(tau, k) * (factorial(N - k) / factorial(N)));
    M.drop(c);
  }
  return true;
}

}  // namespace

int build_mpo_host(int d, int chi, const double* A, const double* B, const double* C,
                   const double* D, int order, double tau_re, double tau_im, int variant,
                   const int* inner_charge, const int* phys_charge, int* w_out, double* W_out,
                   size_t W_capacity, int* level_charge_out, std::string& err) {
  if (!w_out) { err = "mpo_build: w_out is NULL"; return MPOEVO_EINVAL; }
  if (d < 1 || chi < 1) { err = "mpo_build: d and chi must be >= 1"; return MPOEVO_ESHAPE; }
  if (!A || !B || !C || !D) { err = "mpo_build: a Jordan block pointer is NULL"; return MPOEVO_EINVAL; }
  if (order < 1 || order > 4) { err = "mpo_build: order must be 1..4"; return MPOEVO_EINVAL; }
  if (variant != MPOEVO_V1_EXACT && variant != MPOEVO_V2_EXTENDED) { err = "mpo_build: unknown variant"; return MPOEVO_EINVAL; }
  if ((inner_charge == nullptr) != (phys_charge == nullptr)) { err = "mpo_build: give both charge arrays or neither"; return MPOEVO_EINVAL; }
  if (level_charge_out && !inner_charge) { err = "mpo_build: level charges need the input charges"; return MPOEVO_EINVAL; }
  if (!std::isfinite(tau_re) || !std::isfinite(tau_im)) { err = "mpo_build: tau is not finite"; return MPOEVO_ENONFINITE; }
  auto finite = [](const double* p, size_t n) {
    for (size_t i = 0; i < n; ++i) if (!std::isfinite(p[i])) return false;
    return true;
  };
  if (!finite(A, 2ull * chi * chi * d * d) || !finite(B, 2ull * chi * d * d) ||
      !finite(C, 2ull * chi * d * d) || !finite(D, 2ull * d * d)) {
    err = "mpo_build: non-finite entry in the Jordan blocks";
    return MPOEVO_ENONFINITE;
  }
  const Jordan H{d, chi, A, B, C, D};
  const cplx tau(tau_re, tau_im);
  LevelMat M = power_matrix(H, order);
  if (variant == MPOEVO_V2_EXTENDED) extension(M, H, tau);
  fold(M, tau);
  exact_compress(M);
  if (variant == MPOEVO_V2_EXTENDED && !approx_compress(M, tau, err)) return MPOEVO_ESOLVER;

  // Bond layout: (1,...,1) first (code 0 is the smallest code), then increasing codes.
  std::map<int, int> offset;
  int w = 0;
  for (int c : M.present) {
    offset[c] = w;
    w += ipow(chi, decode(c, order).count(2));
  }
  *w_out = w;
  if (level_charge_out) {
    for (int c : M.present) {
      Level l = decode(c, order);
      const int n2 = l.count(2), nv = ipow(chi, n2);
      for (int v = 0; v < nv; ++v) {
        int q = 0, rem = v;
        for (int j = 0; j < n2; ++j) {  // last 2-position is the fastest virtual index
          q += inner_charge[rem % chi];
          rem /= chi;
        }
        level_charge_out[offset[c] + v] = q;
      }
    }
  }
  if (!W_out) return MPOEVO_OK;
  const size_t need = (size_t)w * d * d * w;
  if (W_capacity < need) { err = "mpo_build: W_out capacity too small"; return MPOEVO_ENOMEM; }
  std::memset(W_out, 0, need * 2 * sizeof(double));
  for (auto& kv : M.blk) {
    const int r0 = offset[kv.first.first], c0 = offset[kv.first.second];
    const Tensor4& t = kv.second;
    for (int r = 0; r < t.vr; ++r)
      for (int so = 0; so < d; ++so)
        for (int si = 0; si < d; ++si)
          for (int c = 0; c < t.vc; ++c) {
            const size_t idx = (((size_t)(r0 + r) * d + so) * d + si) * w + (c0 + c);
            W_out[2 * idx] += t.at(r, so, si, c).real();
            W_out[2 * idx + 1] += t.at(r, so, si, c).imag();
          }
  }
  (void)phys_charge;
  return MPOEVO_OK;
}

}  // namespace mpoevo
