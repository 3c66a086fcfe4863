// Fermionic operator strings, region splits with Jordan-Wigner signs, and the
// matrices of site strings in the local basis |0>,|up>,|dn>,|updn>.
//
// Spin-orbital p = 2*orbital + spin (spin 0 = up, 1 = down); the orbitals run
// along the MPS chain, so the Jordan-Wigner order is the chain order and
// |updn> = a+_up a+_dn |0> on every site (the local basis of the Method
// section).
#pragma once
#include <algorithm>
#include <cstdint>
#include <cstring>

#include "common.h"

namespace dmrg {

struct Elem {
  int16_t p = 0;
  int8_t dag = 0;  // 1 = creation
};

// A product of at most four creation/annihilation operators, written left to
// right as an operator product (the rightmost acts first).
struct Str {
  int n = 0;
  Elem e[4];
  void push(int p, int dag) { e[n].p = (int16_t)p; e[n].dag = (int8_t)dag; ++n; }
  int parity() const { return n & 1; }
  QN qn() const {
    QN q;
    for (int k = 0; k < n; ++k) {
      QN d{1, (e[k].p & 1) ? -1 : 1};
      q = e[k].dag ? q + d : q - d;
    }
    return q;
  }
  // 3 bits of length + 9 bits per element (p < 256).
  uint64_t key() const {
    uint64_t k = (uint64_t)n;
    for (int i = 0; i < n; ++i) k |= (uint64_t)(((uint32_t)e[i].p << 1) | (uint32_t)e[i].dag) << (3 + 9 * i);
    return k;
  }
  static Str from_key(uint64_t k) {
    Str s;
    s.n = (int)(k & 7);
    for (int i = 0; i < s.n; ++i) {
      uint32_t v = (uint32_t)((k >> (3 + 9 * i)) & 511);
      s.e[i].p = (int16_t)(v >> 1);
      s.e[i].dag = (int8_t)(v & 1);
    }
    return s;
  }
};

// Canonical order: creators by ascending p, then annihilators by ascending p.
// Only same-kind operators on distinct modes are exchanged, each exchange
// flipping the sign.  Returns the sign (+1/-1), or 0 when a creator or an
// annihilator repeats (the string vanishes).  The input must already have all
// creators left of all annihilators (true for every part of a normal-ordered
// Hamiltonian term split by region).
inline int canonicalize(Str& s) {
  int sign = 1;
  for (int i = 1; i < s.n; ++i) {
    for (int j = i; j > 0; --j) {
      Elem a = s.e[j - 1], b = s.e[j];
      if (a.dag != b.dag) break;  // creators stay left of annihilators
      if (a.p == b.p) return 0;
      if (a.p > b.p) {
        s.e[j - 1] = b;
        s.e[j] = a;
        sign = -sign;
      } else {
        break;
      }
    }
  }
  return sign;
}

// Stable split of a string into consecutive regions (region(p) must be
// non-decreasing in p).  Every exchange of two operators from different
// regions (different modes) flips the sign.  Each part is canonicalised.
// Returns the total sign, 0 if any part vanishes.
template <class RegionFn>
inline int split_regions(const Str& s, RegionFn region, int nreg, Str* parts) {
  int sign = 1;
  for (int i = 0; i < s.n; ++i)
    for (int j = i + 1; j < s.n; ++j)
      if (region(s.e[i].p) > region(s.e[j].p)) sign = -sign;
  for (int r = 0; r < nreg; ++r) parts[r].n = 0;
  for (int i = 0; i < s.n; ++i) {
    Str& P = parts[region(s.e[i].p)];
    P.e[P.n++] = s.e[i];
  }
  for (int r = 0; r < nreg; ++r) {
    int c = canonicalize(parts[r]);
    if (c == 0) return 0;
    sign *= c;
  }
  return sign;
}

// Product of two strings (a then b) in canonical form; sign 0 if it vanishes
// or is not expressible without a creator/annihilator exchange on one mode.
inline int concat_canonical(const Str& a, const Str& b, Str& out) {
  out.n = 0;
  for (int i = 0; i < a.n; ++i) out.e[out.n++] = a.e[i];
  for (int i = 0; i < b.n; ++i) out.e[out.n++] = b.e[i];
  // bring creators left of annihilators: exchanges of distinct modes only
  int sign = 1;
  for (int i = 1; i < out.n; ++i) {
    for (int j = i; j > 0; --j) {
      Elem x = out.e[j - 1], y = out.e[j];
      if (!x.dag && y.dag) {
        if (x.p == y.p) return 0;  // would need the anticommutator
        out.e[j - 1] = y;
        out.e[j] = x;
        sign = -sign;
      } else {
        break;
      }
    }
  }
  int c = canonicalize(out);
  return sign * c;
}

// ---- site matrices --------------------------------------------------------
struct Mat4 {
  double m[4][4];
  static Mat4 zero() { Mat4 r; std::memset(r.m, 0, sizeof(r.m)); return r; }
  static Mat4 eye() { Mat4 r = zero(); for (int i = 0; i < 4; ++i) r.m[i][i] = 1; return r; }
  Mat4 operator*(const Mat4& b) const {
    Mat4 r = zero();
    for (int i = 0; i < 4; ++i)
      for (int k = 0; k < 4; ++k)
        if (m[i][k] != 0)
          for (int j = 0; j < 4; ++j) r.m[i][j] += m[i][k] * b.m[k][j];
    return r;
  }
  bool is_zero() const {
    for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) if (m[i][j] != 0) return false;
    return true;
  }
};

// a+_up: |0>->|up>, |dn>->|updn>;  a+_dn: |0>->|dn>, |up>-> -|updn>.
inline Mat4 site_elem(int spin, int dag) {
  Mat4 c = Mat4::zero();
  if (spin == 0) { c.m[1][0] = 1; c.m[3][2] = 1; }
  else { c.m[2][0] = 1; c.m[3][1] = -1; }
  if (dag) return c;
  Mat4 t = Mat4::zero();
  for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) t.m[i][j] = c.m[j][i];
  return t;
}

// Matrix of a string whose operators all act on one site.
inline Mat4 site_matrix(const Str& s) {
  Mat4 r = Mat4::eye();
  for (int k = 0; k < s.n; ++k) r = r * site_elem(s.e[k].p & 1, s.e[k].dag);
  return r;
}

struct Mat16 {
  double m[16][16];
  static Mat16 zero() { Mat16 r; std::memset(r.m, 0, sizeof(r.m)); return r; }
};

// Matrix of a canonical string on the two window sites (spin-orbitals of the
// first site are 2*i, 2*i+1).  Row/column index n = 4*n1 + n2.  The string is
// split into (site1 part)(site2 part); the second factor passes the
// Jordan-Wigner string of the ket's first site: (-1)^{parity(y2) N(n1)}.
inline Mat16 two_site_matrix(const Str& s, int first_site) {
  Str parts[2];
  int sign = split_regions(s, [&](int p) { return (p >> 1) == first_site ? 0 : 1; }, 2, parts);
  Mat16 r = Mat16::zero();
  if (sign == 0) return r;
  Mat4 y1 = site_matrix(parts[0]), y2 = site_matrix(parts[1]);
  int par2 = parts[1].parity();
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      if (y1.m[a][b] == 0) continue;
      for (int c = 0; c < 4; ++c)
        for (int d = 0; d < 4; ++d) {
          if (y2.m[c][d] == 0) continue;
          double v = sign * y1.m[a][b] * y2.m[c][d];
          if (par2 && (kSiteN[b] & 1)) v = -v;
          r.m[4 * a + c][4 * b + d] += v;
        }
    }
  return r;
}

}  // namespace dmrg
