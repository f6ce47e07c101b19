// Oracle for the sparse wavefunction UCC circuit (Mullinax & Tubman,
// "Large-scale sparse wavefunction circuit simulator for applications with the
// variational quantum eigensolver", arXiv:2301.05726).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
// CPU reference that the HIP library is checked against.  It shares no code,
// header, table or helper with the library; only tests, the smoke check and
// the benchmark's CPU-baseline leg may load it.  The product path never does.
//
// Everything is double precision, single threaded, and uses std::map keyed by
// the determinant bitstring (one bit per spin-orbital, up to 64).  Fermionic
// signs are computed by applying one creation/annihilation operator at a time
// and counting occupied orbitals below the acted-on orbital with a loop.
//
// Conventions (the paper states none of them; these are the readings used by
// the whole project):
//   * |D> = a+_{q1} a+_{q2} ... a+_{qN} |vac>, q1 < q2 < ... < qN;
//   * a_q |D> = (-1)^(#occupied below q) |D - q> if q occupied, else 0;
//     a+_q likewise when q is empty (Jordan-Wigner with Z strings below q);
//   * single  tau_i^a  = a+_a a_i;
//   * double  tau_ij^ab = a+_a a+_b a_j a_i  (i<j, a<b, {i,j} and {a,b} disjoint);
//   * H = sum_{pq,s} h_pq a+_{ps} a_{qs}
//       + 1/2 sum_{pqrs,s,t} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}   (chemist
//     notation, spin-orbital q = 2p + spin), no nuclear repulsion.
//
// Parity pins (tests/): dense Jordan-Wigner statevector with matrix
// exponentials, Hartree-Fock closed form, theta=0 gradient closed form,
// norm preservation, reversibility, central finite differences,
// the variational bound, and literal-vs-Slater-Condon energies.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <utility>
#include <vector>

namespace {

constexpr int OK = 0;
constexpr int EINVAL_ = -1;
constexpr int ECAPACITY_ = -2;
constexpr int EEMPTY_ = -3;

using State = std::map<uint64_t, double>;

// Relative half-width of the "near the cut" window: an amplitude with
// ||c| - thr| <= window * thr after some factor is reported, because a
// different rounding order could flip its truncation decision.
double g_nearcut_window = 1e-3;
// N_MAX / N_CUT truncation (Methods section): when more than g_nmax
// determinants survive a factor, keep the g_ncut largest |c|; 0 = off.
int64_t g_nmax = 0, g_ncut = 0;

// ---------------------------------------------------------------------------
// single fermionic operators (Jordan-Wigner sign by explicit counting)
// ---------------------------------------------------------------------------

int count_below(uint64_t D, int q) {
  int n = 0;
  for (int p = 0; p < q; ++p) n += static_cast<int>((D >> p) & 1u);
  return n;
}

// a_q: returns the sign and updates D, or 0 when q is empty.
int annihilate(uint64_t& D, int q) {
  if (!((D >> q) & 1u)) return 0;
  int s = (count_below(D, q) % 2) ? -1 : 1;
  D &= ~(uint64_t(1) << q);
  return s;
}

// a+_q: returns the sign and updates D, or 0 when q is occupied.
int create(uint64_t& D, int q) {
  if ((D >> q) & 1u) return 0;
  int s = (count_below(D, q) % 2) ? -1 : 1;
  D |= (uint64_t(1) << q);
  return s;
}

struct Exc {
  int i, j, a, b;
  bool dbl;
};

// tau|D> (Eq. 2 excitation operator): operators act right to left.
int apply_tau(const Exc& e, uint64_t D, uint64_t& out) {
  int s = annihilate(D, e.i);
  if (!s) return 0;
  if (e.dbl) {
    int t = annihilate(D, e.j);
    if (!t) return 0;
    s *= t;
    t = create(D, e.b);
    if (!t) return 0;
    s *= t;
  }
  int t = create(D, e.a);
  if (!t) return 0;
  out = D;
  return s * t;
}

// tau^dagger|D> = a+_i a+_j a_b a_a |D>  (single: a+_i a_a |D>).
int apply_tau_dag(const Exc& e, uint64_t D, uint64_t& out) {
  int s = annihilate(D, e.a);
  if (!s) return 0;
  if (e.dbl) {
    int t = annihilate(D, e.b);
    if (!t) return 0;
    s *= t;
    t = create(D, e.j);
    if (!t) return 0;
    s *= t;
  }
  int t = create(D, e.i);
  if (!t) return 0;
  out = D;
  return s * t;
}

int parse_excitations(const int8_t* exc, int64_t M, int nq, std::vector<Exc>& out) {
  out.clear();
  out.reserve(static_cast<size_t>(M));
  for (int64_t k = 0; k < M; ++k) {
    Exc e{exc[4 * k], exc[4 * k + 1], exc[4 * k + 2], exc[4 * k + 3], false};
    bool single = (e.j == -1 && e.b == -1);
    if (single) {
      if (e.i < 0 || e.a < 0 || e.i >= nq || e.a >= nq || e.i == e.a) return EINVAL_;
    } else {
      if (e.i < 0 || e.j < 0 || e.a < 0 || e.b < 0) return EINVAL_;
      if (e.i >= nq || e.j >= nq || e.a >= nq || e.b >= nq) return EINVAL_;
      if (!(e.i < e.j) || !(e.a < e.b)) return EINVAL_;
      if (e.i == e.a || e.i == e.b || e.j == e.a || e.j == e.b) return EINVAL_;
      e.dbl = true;
    }
    out.push_back(e);
  }
  return OK;
}

// ---------------------------------------------------------------------------
// one UCC factor exp(theta (tau - tau^dag))  (Eqs. 3-5)
// ---------------------------------------------------------------------------
// With A = tau - tau^dag and disjoint index sets, A^2 = -1 on every pair
// {L, U} with tau|L> = s|U>, and A = 0 elsewhere, so exp(theta A) acts on a
// pair with amplitudes (x, y) as
//   x' = x cos(theta) - s sin(theta) y,   y' = y cos(theta) + s sin(theta) x.
// This is the closed form the paper takes from the SU(2) treatment of a
// single UCC factor.  The step reads psi and writes a copy.
void apply_factor(const Exc& e, double c, double sn, const State& psi, State& phi) {
  phi = psi;
  for (const auto& kv : psi) {
    const uint64_t D = kv.first;
    const double amp = kv.second;
    uint64_t P = 0;
    int s = apply_tau(e, D, P);
    if (s) {  // D is the lower member of its pair
      auto it = psi.find(P);
      double x = amp;
      double y = (it == psi.end()) ? 0.0 : it->second;
      phi[D] = x * c - s * sn * y;
      phi[P] = y * c + s * sn * x;
      continue;
    }
    int sd = apply_tau_dag(e, D, P);
    if (sd) {  // D is the upper member; the lower member owns the pair if present
      if (psi.count(P)) continue;
      uint64_t chk = 0;
      int sl = apply_tau(e, P, chk);  // sign of tau|L> = s|U>
      double y = amp;
      phi[P] = -sl * sn * y;
      phi[D] = y * c;
    }
  }
}

// Truncation after each factor (Methods section: discard insignificant
// amplitudes after every factor).  Reading: drop |c| < thr (strict), then
// renormalise to unit norm, only if something was dropped.  Returns the norm
// nu used (1 when nothing was dropped) via *nu, the number removed, or EEMPTY.
int prune_renorm(State& phi, double thr, double* nu, int64_t* nearcut) {
  *nu = 1.0;
  if (thr > 0.0 && nearcut) {
    for (const auto& kv : phi)
      if (std::fabs(std::fabs(kv.second) - thr) <= g_nearcut_window * thr) ++*nearcut;
  }
  int64_t removed = 0;
  for (auto it = phi.begin(); it != phi.end();) {
    if (std::fabs(it->second) < thr) {
      it = phi.erase(it);
      ++removed;
    } else {
      ++it;
    }
  }
  if (phi.empty()) return EEMPTY_;
  // N_MAX / N_CUT: order by |c| descending, then determinant ascending (the
  // paper leaves ties open), and keep the first N_CUT.  Two neighbours at the
  // cut closer than the near-cut window (relative) count as a near-cut event.
  if (g_nmax > 0 && static_cast<int64_t>(phi.size()) > g_nmax) {
    std::vector<std::pair<double, uint64_t>> order;
    order.reserve(phi.size());
    for (const auto& kv : phi) order.emplace_back(std::fabs(kv.second), kv.first);
    std::sort(order.begin(), order.end(), [](const std::pair<double, uint64_t>& x, const std::pair<double, uint64_t>& y) {
      return x.first != y.first ? x.first > y.first : x.second < y.second;
    });
    if (nearcut) {
      const double a = order[g_ncut - 1].first, b = order[g_ncut].first;
      if (a - b <= g_nearcut_window * a) ++*nearcut;
    }
    for (size_t i = static_cast<size_t>(g_ncut); i < order.size(); ++i) {
      phi.erase(order[i].second);
      ++removed;
    }
  }
  if (removed) {
    double n2 = 0.0;
    for (const auto& kv : phi) n2 += kv.second * kv.second;
    double n = std::sqrt(n2);
    for (auto& kv : phi) kv.second /= n;
    *nu = n;
  }
  return static_cast<int>(removed > 0);
}

int load_state(int nq, const uint64_t* dets, const double* amps, int64_t n, State& psi) {
  psi.clear();
  for (int64_t k = 0; k < n; ++k) {
    if (nq < 64 && (dets[k] >> nq)) return EINVAL_;
    if (!std::isfinite(amps[k])) return EINVAL_;
    if (!psi.emplace(dets[k], amps[k]).second) return EINVAL_;  // duplicate
  }
  double n2 = 0.0;
  for (const auto& kv : psi) n2 += kv.second * kv.second;
  if (!(n2 > 0.0)) return EINVAL_;
  double nn = std::sqrt(n2);
  for (auto& kv : psi) kv.second /= nn;
  return OK;
}

int check_common(int nq, const double* theta, int64_t M, double thr) {
  if (nq < 2 || nq > 64) return EINVAL_;
  if (!(thr >= 0.0) || !std::isfinite(thr)) return EINVAL_;
  for (int64_t k = 0; k < M; ++k)
    if (!std::isfinite(theta[k])) return EINVAL_;
  return OK;
}

// Forward sweep: psi_k = P_k U_k psi_{k-1} / nu_k for k = 1..M.
// If `keep` is non-null every intermediate state is stored (for the
// gradient), together with nu_k.
int forward(const std::vector<Exc>& ex, const double* theta, double thr, State& psi,
            std::vector<std::vector<std::pair<uint64_t, double>>>* keep, std::vector<double>* nus,
            int64_t* nearcut, int64_t* det_updates) {
  State phi;
  if (keep) keep->emplace_back(psi.begin(), psi.end());
  for (size_t k = 0; k < ex.size(); ++k) {
    if (det_updates) *det_updates += static_cast<int64_t>(psi.size());
    apply_factor(ex[k], std::cos(theta[k]), std::sin(theta[k]), psi, phi);
    double nu = 1.0;
    int r = prune_renorm(phi, thr, &nu, nearcut);
    if (r < 0) return r;
    psi.swap(phi);
    if (keep) keep->emplace_back(psi.begin(), psi.end());
    if (nus) nus->push_back(nu);
  }
  return OK;
}

// ---------------------------------------------------------------------------
// Hamiltonian application
// ---------------------------------------------------------------------------

// Literal second-quantized H|psi>: every term applied operator by operator.
void h_apply_literal(int n, const double* h1, const double* h2, const State& psi, State& out) {
  out.clear();
  const int nq = 2 * n;
  for (const auto& kv : psi) {
    const uint64_t D = kv.first;
    const double c = kv.second;
    for (int sg = 0; sg < 2; ++sg)
      for (int q = 0; q < n; ++q) {
        uint64_t E = D;
        int s1 = annihilate(E, 2 * q + sg);
        if (!s1) continue;
        for (int p = 0; p < n; ++p) {
          uint64_t F = E;
          int s2 = create(F, 2 * p + sg);
          if (!s2) continue;
          out[F] += h1[p * n + q] * s1 * s2 * c;
        }
      }
    // 1/2 (pq|rs) a+_{p sg} a+_{r tu} a_{s tu} a_{q sg}
    for (int sg = 0; sg < 2; ++sg)
      for (int tu = 0; tu < 2; ++tu)
        for (int q = 0; q < n; ++q) {
          uint64_t E1 = D;
          int s1 = annihilate(E1, 2 * q + sg);
          if (!s1) continue;
          for (int s = 0; s < n; ++s) {
            uint64_t E2 = E1;
            int s2 = annihilate(E2, 2 * s + tu);
            if (!s2) continue;
            for (int r = 0; r < n; ++r) {
              uint64_t E3 = E2;
              int s3 = create(E3, 2 * r + tu);
              if (!s3) continue;
              for (int p = 0; p < n; ++p) {
                uint64_t E4 = E3;
                int s4 = create(E4, 2 * p + sg);
                if (!s4) continue;
                double v = h2[((static_cast<size_t>(p) * n + q) * n + r) * n + s];
                out[E4] += 0.5 * v * s1 * s2 * s3 * s4 * c;
              }
            }
          }
        }
  }
  (void)nq;
}

// spin-orbital <pq|rs> = (pr|qs) delta(spin p, spin r) delta(spin q, spin s)
double phys(int n, const double* h2, int p, int q, int r, int s) {
  if ((p & 1) != (r & 1) || (q & 1) != (s & 1)) return 0.0;
  int P = p >> 1, Q = q >> 1, R = r >> 1, S = s >> 1;
  return h2[((static_cast<size_t>(P) * n + R) * n + Q) * n + S];
}
double anti(int n, const double* h2, int p, int q, int r, int s) {
  return phys(n, h2, p, q, r, s) - phys(n, h2, p, q, s, r);
}

// Slater-Condon H|psi> restricted to the support of psi:
//   diagonal   sum_{p in I} h_pp + 1/2 sum_{p,q in I} <pq||pq>
//   single J = e a+_q a_p I:       e [h_qp + sum_{k in I, k != p} <qk||pk>]
//   double J = e a+_q1 a+_q2 a_p2 a_p1 I:  e <q1 q2||p1 p2>
// with the phase e obtained by applying the operators one at a time.
void h_apply_sc(int n, const double* h1, const double* h2, const State& psi, State& out) {
  out.clear();
  const int nq = 2 * n;
  for (const auto& kv : psi) out[kv.first] = 0.0;
  for (const auto& kv : psi) {
    const uint64_t I = kv.first;
    const double c = kv.second;
    std::vector<int> occ, emp;
    for (int q = 0; q < nq; ++q) ((I >> q) & 1u ? occ : emp).push_back(q);
    // diagonal
    double d = 0.0;
    for (int p : occ) d += h1[(p >> 1) * n + (p >> 1)];
    for (int p : occ)
      for (int q : occ) d += 0.5 * anti(n, h2, p, q, p, q);
    out[I] += d * c;
    // singles
    for (int p : occ)
      for (int q : emp) {
        if ((p & 1) != (q & 1)) continue;
        uint64_t J = I;
        int e = annihilate(J, p);
        e *= create(J, q);
        auto it = out.find(J);
        if (it == out.end()) continue;
        double v = h1[(q >> 1) * n + (p >> 1)];
        for (int k : occ)
          if (k != p) v += anti(n, h2, q, k, p, k);
        it->second += e * v * c;
      }
    // doubles
    for (size_t a1 = 0; a1 < occ.size(); ++a1)
      for (size_t a2 = a1 + 1; a2 < occ.size(); ++a2)
        for (size_t b1 = 0; b1 < emp.size(); ++b1)
          for (size_t b2 = b1 + 1; b2 < emp.size(); ++b2) {
            int p1 = occ[a1], p2 = occ[a2], q1 = emp[b1], q2 = emp[b2];
            if (((p1 & 1) + (p2 & 1)) != ((q1 & 1) + (q2 & 1))) continue;
            uint64_t J = I;
            int e = annihilate(J, p1);
            e *= annihilate(J, p2);
            e *= create(J, q2);
            e *= create(J, q1);
            auto it = out.find(J);
            if (it == out.end()) continue;
            it->second += e * anti(n, h2, q1, q2, p1, p2) * c;
          }
  }
}

// Rayleigh quotient <psi|H|psi>/<psi|psi>; `sig` receives H|psi> restricted
// to supp(psi) when non-null.
double energy_of(int mode, int n, const double* h1, const double* h2, const State& psi, State* sig) {
  State hp;
  if (mode == 0)
    h_apply_literal(n, h1, h2, psi, hp);
  else
    h_apply_sc(n, h1, h2, psi, hp);
  double num = 0.0, den = 0.0;
  for (const auto& kv : psi) {
    auto it = hp.find(kv.first);
    double h = (it == hp.end()) ? 0.0 : it->second;
    num += kv.second * h;
    den += kv.second * kv.second;
    if (sig) (*sig)[kv.first] = h;
  }
  return num / den;
}

int write_state(const State& psi, uint64_t* dets, double* amps, int64_t cap, int64_t* n_out) {
  *n_out = static_cast<int64_t>(psi.size());
  if (static_cast<int64_t>(psi.size()) > cap) return ECAPACITY_;
  int64_t k = 0;
  for (const auto& kv : psi) {
    dets[k] = kv.first;
    amps[k] = kv.second;
    ++k;
  }
  return OK;
}

// ---------------------------------------------------------------------------
// which truncation decisions may legitimately differ between two evaluations
// ---------------------------------------------------------------------------
// The cut after every factor (Methods section) compares each amplitude with
// the threshold.  Another evaluation of the same circuit, whose rounding
// differs (another summation order, FP32 amplitudes), may decide differently
// for an amplitude within the near-cut window w*thr of the cut.  Its
// amplitudes then differ from the ones here by up to that amplitude, and
// later factors carry the difference to the pair partners (the descendants
// of the flipped determinant).  This tracks, in exact arithmetic:
//   delta[D]  a bound on |c'_D - c_D| over every such evaluation (c_D = 0 for
//             determinants not held here), apart from a common scale;
//   eps       a bound on the relative difference of that common scale (the
//             runs remove different weights, so they renormalise differently);
// so |c'_D - c_D| <= delta[D] + eps |c_D|.  A decision is uncertain when
// | |phi_D| - thr | <= w thr + delta[D] + eps |phi_D|, phi the state of the
// step before its cut.  Every other decision is the same in both runs, so two
// runs hold the same determinants except those whose decision was uncertain
// at some step.
struct Uncertainty {
  double window = 1e-3;
  std::map<uint64_t, double> delta;
  double eps = 0.0;
  std::vector<std::pair<uint64_t, int64_t>> nearcut;  // (determinant, step): | |phi| - thr | <= w thr
  std::map<uint64_t, int64_t> uncertain;             // determinant -> last step its decision was uncertain
};

double delta_of(const std::map<uint64_t, double>& d, uint64_t key) {
  auto it = d.find(key);
  return it == d.end() ? 0.0 : it->second;
}

// Differences through one factor: on a pair (L, U) the rotation gives
// |dx'| <= |cos| |dx| + |sin| |dy| and |dy'| <= |cos| |dy| + |sin| |dx|, the
// pairs taken whether or not their members are held here.
void propagate_delta(const Exc& e, double c, double sn, std::map<uint64_t, double>& delta) {
  std::map<uint64_t, double> out;
  std::set<uint64_t> lowers;
  for (const auto& kv : delta) {
    uint64_t P = 0;
    if (apply_tau(e, kv.first, P))
      lowers.insert(kv.first);
    else if (apply_tau_dag(e, kv.first, P))
      lowers.insert(P);
    else
      out[kv.first] = kv.second;  // in no pair of this factor
  }
  for (uint64_t L : lowers) {
    uint64_t U = 0;
    apply_tau(e, L, U);
    const double dL = delta_of(delta, L), dU = delta_of(delta, U);
    out[L] = std::fabs(c) * dL + std::fabs(sn) * dU;
    out[U] = std::fabs(c) * dU + std::fabs(sn) * dL;
  }
  delta.swap(out);
}

// The decisions of step `step` on phi (before its cut) and the renormalisation
// that follows; the cut itself is prune_renorm's.
void decide_step(const State& phi, double thr, int64_t step, Uncertainty& u) {
  const double w = u.window * thr;
  std::set<uint64_t> keys;
  for (const auto& kv : phi) keys.insert(kv.first);
  for (const auto& kv : u.delta) keys.insert(kv.first);
  double removed = 0.0;  // weight this run removes
  double rho = 0.0;      // bound on |removed' - removed|
  std::map<uint64_t, double> out;
  for (uint64_t D : keys) {
    auto it = phi.find(D);
    const double v = (it == phi.end()) ? 0.0 : std::fabs(it->second);
    const double dl = delta_of(u.delta, D);
    const double d = dl + u.eps * v;  // bound on the other run's difference here
    if (it != phi.end() && std::fabs(v - thr) <= w) u.nearcut.emplace_back(D, step);
    if (v < thr) removed += v * v;
    double nd;
    if (std::fabs(v - thr) <= w + d) {  // either decision possible
      u.uncertain[D] = step;
      nd = (v >= thr) ? std::max(v, d) : v + d;  // kept here: 0 or within d; cut here: up to v + d there
      rho += (v + d) * (v + d);
    } else if (v < thr) {  // both runs cut
      nd = 0.0;
      rho += 4.0 * (v + d) * d;
    } else {  // both runs keep
      nd = dl;
    }
    if (nd > 0.0) out[D] = nd;
  }
  u.delta.swap(out);
  if (rho > 0.0 || removed > 0.0) {
    // nu^2 = 1 - removed for both runs (unit-norm states before the step), so
    // |nu / nu' - 1| <= rho / (1 - removed - rho)
    const double nu = std::sqrt(1.0 - removed);
    const double es = rho / (1.0 - removed - rho);
    for (auto& kv : u.delta) kv.second *= (1.0 + es) / nu;
    u.eps = u.eps * (1.0 + es) + es;
  }
}

}  // namespace

extern "C" {

void orc_set_nearcut_window(double rel) { g_nearcut_window = rel; }

// N_MAX / N_CUT truncation for every later call (0, 0 turns it off).
int orc_set_topk(int64_t n_max, int64_t n_cut) {
  if (n_max == 0 && n_cut == 0) {
    g_nmax = g_ncut = 0;
    return OK;
  }
  if (n_cut < 1 || n_cut > n_max) return EINVAL_;
  g_nmax = n_max;
  g_ncut = n_cut;
  return OK;
}

// tau|D> for one excitation row (i, j, a, b): sign in {-1, 0, +1}.
int orc_tau(const int8_t* exc4, uint64_t D, uint64_t* out) {
  Exc e{exc4[0], exc4[1], exc4[2], exc4[3], !(exc4[1] == -1 && exc4[3] == -1)};
  uint64_t r = 0;
  int s = apply_tau(e, D, r);
  *out = r;
  return s;
}

// Forward circuit (Eq. 3) with per-factor truncation.  The initial state is
// normalised first.  Output sorted by determinant.
int orc_apply_ucc(int nq, const uint64_t* dets0, const double* amps0, int64_t n0, const int8_t* exc,
                  const double* theta, int64_t M, double thr, uint64_t* dets_out, double* amps_out,
                  int64_t cap, int64_t* n_out, int64_t* nearcut, int64_t* det_updates) {
  int r = check_common(nq, theta, M, thr);
  if (r) return r;
  std::vector<Exc> ex;
  if ((r = parse_excitations(exc, M, nq, ex))) return r;
  State psi;
  if ((r = load_state(nq, dets0, amps0, n0, psi))) return r;
  int64_t nc = 0, du = 0;
  r = forward(ex, theta, thr, psi, nullptr, nullptr, &nc, &du);
  if (nearcut) *nearcut = nc;
  if (det_updates) *det_updates = du;
  if (r) return r;
  return write_state(psi, dets_out, amps_out, cap, n_out);
}

// The forward circuit with the analysis above: the near-cut events (every
// determinant and step with | |phi| - thr | <= window thr), the determinants
// whose decision was uncertain at some step (with the last such step), and
// the final bounds delta (determinant, bound) and eps.  The final state is
// orc_apply_ucc's.  Not defined with N_MAX / N_CUT on (EINVAL).  Each list
// is written up to its capacity; ECAPACITY (with the counts set) when one is
// longer.
int orc_uncertainty(int nq, const uint64_t* dets0, const double* amps0, int64_t n0, const int8_t* exc,
                    const double* theta, int64_t M, double thr, double window, uint64_t* nc_key, int64_t* nc_step,
                    int64_t nc_cap, int64_t* nc_n, uint64_t* un_key, int64_t* un_step, int64_t un_cap,
                    int64_t* un_n, uint64_t* dl_key, double* dl_val, int64_t dl_cap, int64_t* dl_n,
                    double* eps_out) {
  int r = check_common(nq, theta, M, thr);
  if (r) return r;
  if (g_nmax > 0 || !(window >= 0.0)) return EINVAL_;
  std::vector<Exc> ex;
  if ((r = parse_excitations(exc, M, nq, ex))) return r;
  State psi;
  if ((r = load_state(nq, dets0, amps0, n0, psi))) return r;
  Uncertainty u;
  u.window = window;
  State phi;
  for (int64_t k = 0; k < M; ++k) {
    const double c = std::cos(theta[k]), sn = std::sin(theta[k]);
    apply_factor(ex[static_cast<size_t>(k)], c, sn, psi, phi);
    if (thr > 0.0) {
      propagate_delta(ex[static_cast<size_t>(k)], c, sn, u.delta);
      decide_step(phi, thr, k + 1, u);
    }
    double nu = 1.0;
    if ((r = prune_renorm(phi, thr, &nu, nullptr)) < 0) return r;
    psi.swap(phi);
  }
  *nc_n = static_cast<int64_t>(u.nearcut.size());
  *un_n = static_cast<int64_t>(u.uncertain.size());
  *dl_n = static_cast<int64_t>(u.delta.size());
  *eps_out = u.eps;
  if (*nc_n > nc_cap || *un_n > un_cap || *dl_n > dl_cap) return ECAPACITY_;
  for (size_t i = 0; i < u.nearcut.size(); ++i) {
    nc_key[i] = u.nearcut[i].first;
    nc_step[i] = u.nearcut[i].second;
  }
  int64_t i = 0;
  for (const auto& kv : u.uncertain) {
    un_key[i] = kv.first;
    un_step[i++] = kv.second;
  }
  i = 0;
  for (const auto& kv : u.delta) {
    dl_key[i] = kv.first;
    dl_val[i++] = kv.second;
  }
  return OK;
}

// Wavefunction entropy (Eq. 6): S = -sum_I p_I ln p_I with p_I = c_I^2 / sum c^2
// (terms with c_I = 0 contribute 0), of the initial state and after every
// factor of the truncated forward circuit: S_out[0..M].
int orc_entropy_trajectory(int nq, const uint64_t* dets0, const double* amps0, int64_t n0, const int8_t* exc,
                           const double* theta, int64_t M, double thr, double* S_out) {
  int r = check_common(nq, theta, M, thr);
  if (r) return r;
  std::vector<Exc> ex;
  if ((r = parse_excitations(exc, M, nq, ex))) return r;
  State psi;
  if ((r = load_state(nq, dets0, amps0, n0, psi))) return r;
  auto entropy = [](const State& st) {
    double n2 = 0.0;
    for (const auto& kv : st) n2 += kv.second * kv.second;
    double S = 0.0;
    for (const auto& kv : st) {
      const double p = kv.second * kv.second / n2;
      if (p > 0.0) S -= p * std::log(p);
    }
    return S;
  };
  S_out[0] = entropy(psi);
  State phi;
  for (int64_t k = 0; k < M; ++k) {
    apply_factor(ex[k], std::cos(theta[k]), std::sin(theta[k]), psi, phi);
    double nu = 1.0;
    if ((r = prune_renorm(phi, thr, &nu, nullptr)) < 0) return r;
    psi.swap(phi);
    S_out[k + 1] = entropy(psi);
  }
  return OK;
}

// Number of determinants the sparse state holds: initially, and after each
// factor with its truncation (Eq. 3 applied in order): n_out[0..M].
int orc_live_trajectory(int nq, const uint64_t* dets0, const double* amps0, int64_t n0, const int8_t* exc,
                        const double* theta, int64_t M, double thr, int64_t* n_out) {
  int r = check_common(nq, theta, M, thr);
  if (r) return r;
  std::vector<Exc> ex;
  if ((r = parse_excitations(exc, M, nq, ex))) return r;
  State psi;
  if ((r = load_state(nq, dets0, amps0, n0, psi))) return r;
  n_out[0] = static_cast<int64_t>(psi.size());
  State phi;
  for (int64_t k = 0; k < M; ++k) {
    apply_factor(ex[k], std::cos(theta[k]), std::sin(theta[k]), psi, phi);
    double nu = 1.0;
    if ((r = prune_renorm(phi, thr, &nu, nullptr)) < 0) return r;
    psi.swap(phi);
    n_out[k + 1] = static_cast<int64_t>(psi.size());
  }
  return OK;
}

// Energy <psi|H|psi>/<psi|psi> of a given state; mode 0 literal, 1 Slater-Condon.
int orc_energy(int mode, int n_orb, const double* h1, const double* h2, const uint64_t* dets,
               const double* amps, int64_t n, double* E) {
  State psi;
  for (int64_t k = 0; k < n; ++k) psi[dets[k]] = amps[k];
  if (psi.empty()) return EEMPTY_;
  *E = energy_of(mode, n_orb, h1, h2, psi, nullptr);
  return OK;
}

// H|psi> restricted to supp(psi) (Slater-Condon, mode 1, or literal, mode 0).
int orc_h_apply(int mode, int n_orb, const double* h1, const double* h2, const uint64_t* dets,
                const double* amps, int64_t n, double* out) {
  State psi, hp;
  for (int64_t k = 0; k < n; ++k) psi[dets[k]] = amps[k];
  if (mode == 0)
    h_apply_literal(n_orb, h1, h2, psi, hp);
  else
    h_apply_sc(n_orb, h1, h2, psi, hp);
  for (int64_t k = 0; k < n; ++k) {
    auto it = hp.find(dets[k]);
    out[k] = (it == hp.end()) ? 0.0 : it->second;
  }
  return OK;
}

// E(theta) = forward sweep + Slater-Condon energy.
int orc_energy_theta(int nq, const uint64_t* dets0, const double* amps0, int64_t n0, const int8_t* exc,
                     const double* theta, int64_t M, double thr, const double* h1, const double* h2,
                     int mode, double* E) {
  int r = check_common(nq, theta, M, thr);
  if (r) return r;
  std::vector<Exc> ex;
  if ((r = parse_excitations(exc, M, nq, ex))) return r;
  State psi;
  if ((r = load_state(nq, dets0, amps0, n0, psi))) return r;
  if ((r = forward(ex, theta, thr, psi, nullptr, nullptr, nullptr, nullptr))) return r;
  *E = energy_of(mode, nq / 2, h1, h2, psi, nullptr);
  return OK;
}

// Energy and exact gradient with the truncation decisions held fixed.
// psi_k = P_k U_k psi_{k-1} / nu_k; E = <psi_M|H|psi_M>.
// lambda_M = P_M (H - E) psi_M; for k = M..1:
//   w = U_k^T lambda_k;  g_k = (2/nu_k) <w|A_k psi_{k-1}>;  lambda_{k-1} = P_{k-1} w / nu_k.
// At threshold 0 this is dE/dtheta_k = 2 <(H-E) psi| A_k-propagated psi>.
int orc_energy_and_grad(int nq, const uint64_t* dets0, const double* amps0, int64_t n0,
                        const int8_t* exc, const double* theta, int64_t M, double thr, const double* h1,
                        const double* h2, int mode, double* E, double* grad, int64_t* nearcut) {
  int r = check_common(nq, theta, M, thr);
  if (r) return r;
  std::vector<Exc> ex;
  if ((r = parse_excitations(exc, M, nq, ex))) return r;
  State psi;
  if ((r = load_state(nq, dets0, amps0, n0, psi))) return r;
  std::vector<std::vector<std::pair<uint64_t, double>>> states;
  std::vector<double> nus;
  int64_t nc = 0;
  r = forward(ex, theta, thr, psi, &states, &nus, &nc, nullptr);
  if (nearcut) *nearcut = nc;
  if (r) return r;
  State sig;
  const int n = nq / 2;
  double e = energy_of(mode, n, h1, h2, psi, &sig);
  *E = e;
  State lam;
  for (const auto& kv : psi) lam[kv.first] = sig[kv.first] - e * kv.second;
  State w;
  for (int64_t k = M; k >= 1; --k) {
    const Exc& ek = ex[static_cast<size_t>(k - 1)];
    const double th = theta[k - 1];
    apply_factor(ek, std::cos(-th), std::sin(-th), lam, w);  // U_k^T = U_k(-theta)
    const auto& prev = states[static_cast<size_t>(k - 1)];
    double dot = 0.0;
    for (const auto& kv : prev) {
      uint64_t P = 0;
      int s = apply_tau(ek, kv.first, P);
      if (s) {
        auto it = w.find(P);
        if (it != w.end()) dot += s * kv.second * it->second;
      }
      s = apply_tau_dag(ek, kv.first, P);
      if (s) {
        auto it = w.find(P);
        if (it != w.end()) dot -= s * kv.second * it->second;
      }
    }
    const double nu = nus[static_cast<size_t>(k - 1)];
    grad[k - 1] = 2.0 * dot / nu;
    lam.clear();
    for (const auto& kv : prev) {
      auto it = w.find(kv.first);
      lam[kv.first] = (it == w.end()) ? 0.0 : it->second / nu;
    }
  }
  return OK;
}

// Central finite differences dE/dtheta_p = (E(theta + h e_p) - E(theta - h e_p)) / 2h
// for the listed parameter indices.
int orc_fd_grad(int nq, const uint64_t* dets0, const double* amps0, int64_t n0, const int8_t* exc,
                const double* theta, int64_t M, double thr, const double* h1, const double* h2, int mode,
                double h, const int64_t* idx, int64_t n_idx, double* out) {
  std::vector<double> t(theta, theta + M);
  for (int64_t q = 0; q < n_idx; ++q) {
    const int64_t p = idx[q];
    if (p < 0 || p >= M) return EINVAL_;
    double ep = 0.0, em = 0.0;
    t[p] = theta[p] + h;
    int r = orc_energy_theta(nq, dets0, amps0, n0, exc, t.data(), M, thr, h1, h2, mode, &ep);
    if (r) return r;
    t[p] = theta[p] - h;
    r = orc_energy_theta(nq, dets0, amps0, n0, exc, t.data(), M, thr, h1, h2, mode, &em);
    if (r) return r;
    t[p] = theta[p];
    out[q] = (ep - em) / (2.0 * h);
  }
  return OK;
}

// Reverse circuit: applies U_M(-theta_M) ... U_1(-theta_1) to a state with
// no truncation; with a forward sweep at threshold 0 this returns psi_0.
int orc_apply_inverse(int nq, const uint64_t* dets0, const double* amps0, int64_t n0, const int8_t* exc,
                      const double* theta, int64_t M, uint64_t* dets_out, double* amps_out, int64_t cap,
                      int64_t* n_out) {
  int r = check_common(nq, theta, M, 0.0);
  if (r) return r;
  std::vector<Exc> ex;
  if ((r = parse_excitations(exc, M, nq, ex))) return r;
  State psi, phi;
  for (int64_t k = 0; k < n0; ++k) psi[dets0[k]] = amps0[k];
  for (int64_t k = M - 1; k >= 0; --k) {
    apply_factor(ex[static_cast<size_t>(k)], std::cos(-theta[k]), std::sin(-theta[k]), psi, phi);
    psi.swap(phi);
  }
  return write_state(psi, dets_out, amps_out, cap, n_out);
}

}  // extern "C"
