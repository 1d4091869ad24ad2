// Host assembly of the Q1 Helmholtz matrices (paper Sec. 3.2: finite-element
// discretisation of the Helmholtz equation on the compartment mesh).
//
// Rows are assembled independently (row i gathers the element rows of the
// hexahedra around node i, in ascending element id), which parallelises over
// threads without write conflicts and sums every entry (i,j) and (j,i) from
// the same terms in the same order: K, M, M_eta and the wall masses come out
// bitwise symmetric.
#include <algorithm>
#include <cstdarg>
#include <thread>
#include <unordered_map>

#include "ctx.h"
#include "p1.h"
#include "q1.h"

namespace {

template <class F>
void parallel_for(int64_t n, F f) {
  unsigned hc = std::thread::hardware_concurrency();
  int nt = int(hc == 0 ? 1 : (hc > 16 ? 16 : hc));
  if (n < 20000 || nt == 1) {
    f(int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    int64_t b = t * chunk, e = std::min(n, b + chunk);
    if (b >= e) break;
    th.emplace_back([=, &f] { f(b, e); });
  }
  for (auto& x : th) x.join();
}

inline int64_t find_col(const HostAsm& a, int32_t row, int32_t col) {
  const int32_t* b = a.col.data() + a.rowptr[row];
  const int32_t* e = a.col.data() + a.rowptr[row + 1];
  const int32_t* p = std::lower_bound(b, e, col);
  if (p == e || *p != col) return -1;
  return p - a.col.data();
}

void gather_elem(const HostAsm& a, int32_t e, double X[8][3]) {
  for (int l = 0; l < a.npe; ++l) {
    int32_t v = a.hex[int64_t(e) * a.npe + l];
    for (int d = 0; d < 3; ++d) X[l][d] = a.xyz[int64_t(v) * 3 + d];
  }
}

void assemble_rows(HostAsm& a, const double* eta, bool km) {
  parallel_for(a.n, [&](int64_t r0, int64_t r1) {
    for (int64_t i = r0; i < r1; ++i) {
      for (int64_t q = a.rowptr[i]; q < a.rowptr[i + 1]; ++q) {
        if (km) { a.K[q] = 0.0; a.M[q] = 0.0; }
        if (eta) a.Meta[q] = 0.0;
      }
      for (int64_t t = a.n2e_ptr[i]; t < a.n2e_ptr[i + 1]; ++t) {
        int32_t e = a.n2e[t];
        int loc = -1;
        for (int l = 0; l < a.npe; ++l)
          if (a.hex[int64_t(e) * a.npe + l] == int32_t(i)) { loc = l; break; }
        double X[8][3], Kr[8], Mr[8];
        gather_elem(a, e, X);
        if (a.npe == 8) {
          q1::hex_rows(X, loc, Kr, Mr);
        } else {
          double T[4][3];
          for (int l = 0; l < 4; ++l)
            for (int d = 0; d < 3; ++d) T[l][d] = X[l][d];
          p1::tet_rows(T, loc, Kr, Mr);
        }
        for (int b = 0; b < a.npe; ++b) {
          int64_t pos = find_col(a, int32_t(i), a.hex[int64_t(e) * a.npe + b]);
          if (km) { a.K[pos] += Kr[b]; a.M[pos] += Mr[b]; }
          if (eta) a.Meta[pos] += eta[e] * Mr[b];
        }
      }
    }
  });
}

}  // namespace

int mesh_pattern(int64_t n, int64_t ne, int npe, const int32_t* hex, std::vector<int64_t>* n2e_ptr_out,
                 std::vector<int32_t>* n2e_out, std::vector<int64_t>* rowptr_out, std::vector<int32_t>* col_out) {
  // node -> element adjacency, ascending element id
  std::vector<int64_t>& n2e_ptr = *n2e_ptr_out;
  std::vector<int32_t>& n2e = *n2e_out;
  n2e_ptr.assign(n + 1, 0);
  for (int64_t q = 0; q < ne * npe; ++q) n2e_ptr[hex[q] + 1]++;
  for (int64_t i = 0; i < n; ++i) n2e_ptr[i + 1] += n2e_ptr[i];
  n2e.assign(n2e_ptr[n], 0);
  {
    std::vector<int64_t> fill(n2e_ptr.begin(), n2e_ptr.end() - 1);
    for (int64_t e = 0; e < ne; ++e)
      for (int l = 0; l < npe; ++l) n2e[fill[hex[e * npe + l]]++] = int32_t(e);
  }
  for (int64_t i = 0; i < n; ++i)
    if (n2e_ptr[i + 1] == n2e_ptr[i])
      return hz_fail(HZ_ERR_INVALID, "hz_assemble: node %lld belongs to no element", (long long)i);

  // CSR pattern: union of the nodes of the elements around each node
  std::vector<int32_t> cnt(n);
  auto row_nodes = [&](int64_t i, int32_t* buf) {
    int c = 0;
    for (int64_t t = n2e_ptr[i]; t < n2e_ptr[i + 1]; ++t)
      for (int l = 0; l < npe; ++l) buf[c++] = hex[int64_t(n2e[t]) * npe + l];
    std::sort(buf, buf + c);
    return int(std::unique(buf, buf + c) - buf);
  };
  int64_t maxdeg = 0;
  for (int64_t i = 0; i < n; ++i) maxdeg = std::max(maxdeg, n2e_ptr[i + 1] - n2e_ptr[i]);
  parallel_for(n, [&](int64_t r0, int64_t r1) {
    std::vector<int32_t> buf(maxdeg * npe);
    for (int64_t i = r0; i < r1; ++i) cnt[i] = row_nodes(i, buf.data());
  });
  std::vector<int64_t>& rowptr = *rowptr_out;
  rowptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) rowptr[i + 1] = rowptr[i] + cnt[i];
  if (rowptr[n] >= (int64_t(1) << 31) - (n * 64))
    return hz_fail(HZ_ERR_INVALID, "hz_assemble: %lld nonzeros exceed the int32 index range", (long long)rowptr[n]);
  col_out->assign(rowptr[n], 0);
  parallel_for(n, [&](int64_t r0, int64_t r1) {
    std::vector<int32_t> buf(maxdeg * npe);
    for (int64_t i = r0; i < r1; ++i) {
      int c = row_nodes(i, buf.data());
      std::copy(buf.data(), buf.data() + c, col_out->data() + rowptr[i]);
    }
  });
  return HZ_OK;
}

int host_assemble_meta(HostAsm* a, const double* eta) {
  if (!eta) {
    a->Meta.clear();
    return HZ_OK;
  }
  for (int64_t e = 0; e < a->ne; ++e)
    if (!std::isfinite(eta[e])) return hz_fail(HZ_ERR_INVALID, "eta[%lld] is not finite", (long long)e);
  a->Meta.assign(a->col.size(), 0.0);
  assemble_rows(*a, eta, false);
  return HZ_OK;
}

int host_assemble(const hz_mesh* m, const double* eta, HostAsm* out, int ntags, std::vector<int32_t>* perm) {
  HostAsm& a = *out;
  a.ntags = ntags;
  if (!m || !m->xyz || !m->hex || m->n_nodes <= 0 || m->n_elems <= 0 || m->n_bfaces < 0 ||
      (m->n_bfaces > 0 && (!m->bface || !m->bface_tag || !m->bface_src)))
    return hz_fail(HZ_ERR_INVALID, "hz_assemble: null or empty mesh arrays");
  if (m->elem_type != HZ_HEX8 && m->elem_type != HZ_TET4)
    return hz_fail(HZ_ERR_INVALID, "hz_assemble: unknown element type %d", m->elem_type);
  if (m->src_kind != HZ_SRC_NEUMANN && m->src_kind != HZ_SRC_DIRICHLET)
    return hz_fail(HZ_ERR_INVALID, "hz_assemble: unknown source kind %d", m->src_kind);
  if (m->fe_scheme != HZ_GALERKIN && m->fe_scheme != HZ_GLS)
    return hz_fail(HZ_ERR_INVALID, "hz_assemble: unknown finite-element scheme %d", m->fe_scheme);
  a.npe = m->elem_type == HZ_TET4 ? 4 : 8;
  a.npf = m->elem_type == HZ_TET4 ? 3 : 4;
  a.n = m->n_nodes;
  a.ne = m->n_elems;
  a.nb = m->n_bfaces;
  a.xyz.assign(m->xyz, m->xyz + int64_t(a.n) * 3);
  a.hex.assign(m->hex, m->hex + int64_t(a.ne) * a.npe);
  for (double v : a.xyz)
    if (!std::isfinite(v)) return hz_fail(HZ_ERR_INVALID, "hz_assemble: non-finite coordinate");
  for (int32_t v : a.hex)
    if (v < 0 || v >= a.n) return hz_fail(HZ_ERR_INVALID, "hz_assemble: element node %d out of range", v);
  if (a.nb > 0) {
    a.bface.assign(m->bface, m->bface + int64_t(a.nb) * a.npf);
    a.btag.assign(m->bface_tag, m->bface_tag + a.nb);
    a.bsrc.assign(m->bface_src, m->bface_src + a.nb);
    for (int32_t v : a.bface)
      if (v < 0 || v >= a.n) return hz_fail(HZ_ERR_INVALID, "hz_assemble: face node %d out of range", v);
    for (int32_t t : a.btag)
      if (t < 0 || t >= ntags) return hz_fail(HZ_ERR_INVALID, "hz_assemble: wall tag %d not in 0..%d", t, ntags - 1);
  }

  HZ_TRY(mesh_pattern(a.n, a.ne, a.npe, a.hex.data(), &a.n2e_ptr, &a.n2e, &a.rowptr, &a.col));
  if (perm && (m->order == HZ_ORDER_RCM || m->sigma > 0)) {
    // renumber the nodes (internal p = mesh node perm[p]) and rebuild the pattern
    node_order(a.n, a.rowptr, a.col, m->order, m->sigma, perm);
    std::vector<int32_t> iperm(a.n);
    for (int64_t p = 0; p < a.n; ++p) iperm[(*perm)[p]] = int32_t(p);
    for (int64_t p = 0; p < a.n; ++p)
      for (int d = 0; d < 3; ++d) a.xyz[p * 3 + d] = m->xyz[int64_t((*perm)[p]) * 3 + d];
    for (int32_t& v : a.hex) v = iperm[v];
    for (int32_t& v : a.bface) v = iperm[v];
    HZ_TRY(mesh_pattern(a.n, a.ne, a.npe, a.hex.data(), &a.n2e_ptr, &a.n2e, &a.rowptr, &a.col));
  } else if (perm) {
    perm->clear();
  }
  a.diag.assign(a.n, -1);
  for (int64_t i = 0; i < a.n; ++i) a.diag[i] = find_col(a, int32_t(i), int32_t(i));

  // values
  a.K.assign(a.col.size(), 0.0);
  a.M.assign(a.col.size(), 0.0);
  if (eta) {
    for (int64_t e = 0; e < a.ne; ++e)
      if (!std::isfinite(eta[e])) return hz_fail(HZ_ERR_INVALID, "eta[%lld] is not finite", (long long)e);
    a.Meta.assign(a.col.size(), 0.0);
  }
  assemble_rows(a, eta, true);
  for (int64_t i = 0; i < a.n; ++i)
    if (!(a.K[a.diag[i]] > 0.0) || !(a.M[a.diag[i]] > 0.0))
      return hz_fail(HZ_ERR_INVALID, "hz_assemble: degenerate element at node %lld (inverted or flat)",
                     (long long)i);

  // wall boundary masses: entry slots in CSR order of first touch by the faces
  std::unordered_map<int64_t, int32_t> slot;
  a.bpos.clear();
  a.bmass.clear();
  std::map<int64_t, double> patch;   // (row * n + col) -> value
  for (int64_t f = 0; f < a.nb; ++f) {
    const int nf = a.npf;
    double X[4][3], Fe[4][4];
    for (int l = 0; l < nf; ++l)
      for (int d = 0; d < 3; ++d) X[l][d] = a.xyz[int64_t(a.bface[f * nf + l]) * 3 + d];
    if (nf == 4) {
      q1::quad_mass(X, Fe);
    } else {
      double T[3][3], F3[3][3];
      for (int l = 0; l < 3; ++l)
        for (int d = 0; d < 3; ++d) T[l][d] = X[l][d];
      p1::tri_mass(T, F3);
      for (int l = 0; l < 3; ++l)
        for (int o = 0; o < 3; ++o) Fe[l][o] = F3[l][o];
    }
    for (int l = 0; l < nf; ++l)
      for (int o = 0; o < nf; ++o) {
        int32_t r = a.bface[f * nf + l], c = a.bface[f * nf + o];
        int64_t pos = find_col(a, r, c);
        if (pos < 0) return hz_fail(HZ_ERR_INVALID, "hz_assemble: boundary face %lld is not an element face", (long long)f);
        auto it = slot.find(pos);
        int32_t s;
        if (it == slot.end()) {
          s = int32_t(a.bpos.size());
          slot.emplace(pos, s);
          a.bpos.push_back(pos);
          a.bmass.insert(a.bmass.end(), ntags, 0.0);
        } else {
          s = it->second;
        }
        a.bmass[int64_t(s) * ntags + a.btag[f]] += Fe[l][o];
        if (a.bsrc[f]) patch[int64_t(r) * a.n + c] += Fe[l][o];
      }
  }
  // patch CSR over its rows
  a.prow.clear(); a.pptr.assign(1, 0); a.pcol.clear(); a.pval.clear();
  int64_t last = -1;
  for (auto& kv : patch) {
    int64_t r = kv.first / a.n;
    if (r != last) {
      if (last >= 0) a.pptr.push_back(int32_t(a.pcol.size()));
      a.prow.push_back(int32_t(r));
      last = r;
    }
    a.pcol.push_back(int32_t(kv.first % a.n));
    a.pval.push_back(kv.second);
  }
  if (last >= 0) a.pptr.push_back(int32_t(a.pcol.size()));
  // Dirichlet set: the nodes of the source faces
  a.dir.clear();
  if (m->src_kind == HZ_SRC_DIRICHLET) {
    a.dir.assign(a.n, 0);
    for (int64_t f = 0; f < a.nb; ++f)
      if (a.bsrc[f])
        for (int l = 0; l < a.npf; ++l) a.dir[a.bface[f * a.npf + l]] = 1;
  }
  // GLS element size: the mean edge length (hexahedra: the 12 pairs of
  // tensor corners that differ in one index; tetrahedra: the 6 vertex pairs)
  a.gls_h = 0.0;
  if (m->fe_scheme == HZ_GLS) {
    double sum = 0.0;
    int64_t cnt = 0;
    auto edge = [&](int32_t u, int32_t v) {
      double d2 = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double t = a.xyz[int64_t(u) * 3 + d] - a.xyz[int64_t(v) * 3 + d];
        d2 += t * t;
      }
      sum += std::sqrt(d2);
      ++cnt;
    };
    for (int64_t e = 0; e < a.ne; ++e) {
      const int32_t* v = &a.hex[e * a.npe];
      if (a.npe == 8) {
        for (int bit = 1; bit < 8; bit <<= 1)
          for (int c = 0; c < 8; ++c)
            if (!(c & bit)) edge(v[c], v[c | bit]);
      } else {
        for (int c = 0; c < 4; ++c)
          for (int d = c + 1; d < 4; ++d) edge(v[c], v[d]);
      }
    }
    a.gls_h = sum / double(std::max<int64_t>(cnt, 1));
  }
  return HZ_OK;
}

void build_sell(const HostAsm& a, int64_t nrows, SellHost* s) {
  s->n_rows = int32_t(nrows);
  s->n_slices = ceil_div(nrows, kWave);
  s->ptr.assign(int64_t(s->n_slices) + 1, 0);
  for (int32_t sl = 0; sl < s->n_slices; ++sl) {
    int64_t w = 0;
    for (int l = 0; l < kWave; ++l) {
      int64_t i = int64_t(sl) * kWave + l;
      if (i < a.n) w = std::max(w, a.rowptr[i + 1] - a.rowptr[i]);
    }
    s->ptr[sl + 1] = s->ptr[sl] + int32_t(w * kWave);
  }
  s->n_pad = s->ptr[s->n_slices];
  s->col.assign(s->n_pad, 0);
  s->src.assign(s->n_pad, -1);
  for (int32_t sl = 0; sl < s->n_slices; ++sl) {
    int64_t w = (s->ptr[sl + 1] - s->ptr[sl]) / kWave;
    for (int l = 0; l < kWave; ++l) {
      int64_t i = int64_t(sl) * kWave + l;
      for (int64_t k = 0; k < w; ++k) {
        int64_t p = s->ptr[sl] + k * kWave + l;
        if (i >= a.n) {
          s->col[p] = 0;
        } else if (a.rowptr[i] + k < a.rowptr[i + 1]) {
          s->col[p] = a.col[a.rowptr[i] + k];
          s->src[p] = a.rowptr[i] + k;
        } else {
          s->col[p] = int32_t(i);
        }
      }
    }
  }
}
