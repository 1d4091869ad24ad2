// Non-overlapping Schwarz domain decomposition with Robin transmission
// conditions (paper Sec. 4, domain-decomposition part: absorbing
// transmission conditions on the interfaces; the subdomain solves run on the
// GPU at every interface iteration).
//
// Structured partition of a box mesh into px x py x pz subdomains along
// element planes (cut of axis d for part a at element (a n_d) / p_d).  Each
// subdomain s has its own Q1 operator (its elements and wall faces) plus the
// Robin term alpha_st M_G on every interface face set G_st:
//     (A~_s + sum_t alpha_st M_Gst) u_s = f_s + sum_t R_st^T lam_st,
// two-sided: alpha_st = a_lo when s is the lower-index side of G_st (its
// face on the high side of an axis), a_hi when it is the higher-index side;
// with f_s = (R_s f) / multiplicity.  All subdomain systems are stacked into
// one block-diagonal sliced-ELL system whose blocks are the segments of the
// segmented Krylov solvers: one batched solve advances every subdomain in
// lock-step with its own Krylov scalars.  One multiplier vector lives on the
// nodes of each ordered face-neighbour pair (cross points included) and is
// updated by
//     lam_st <- (T_st + T_ts) R_ts u_t - lam_ts = (a_lo + a_hi) M_Gst R_ts u_t - lam_ts.
// The fixed point of this map (the interface system (I - B) lam = c) is
// solved by restarted GMRES in complex128 (or iterated plainly on request);
// the glued solution (average of duplicated interface values) is then
// checked against the global FP64 residual.
#include <algorithm>
#include <chrono>
#include <complex>
#include <map>

#include "ops.h"
#include "q1.h"
#include "solve.h"

namespace {

constexpr int NTAG = 12;   // 6 walls + interface towards the low/high side of each axis

struct DDSub {
  int lo[3], ln[3];
  int64_t n = 0, nrows = 0, row_off = 0;
  std::vector<int32_t> l2g;
  HostAsm a;
};

struct DDPair {
  int s, t, tag;
  std::vector<int32_t> g;            // global node ids of G_st, ascending
  std::vector<int32_t> ins, int_;    // local ids in s and in t
  std::vector<int32_t> mptr, mcol;   // face mass over G (pair-local indices)
  std::vector<double> mval;
};

struct DDData {
  int parts[3] = {1, 1, 1};
  int nsub = 0;
  std::vector<DDSub> subs;
  std::vector<DDPair> pairs;
  std::vector<int64_t> lam_off;
  int64_t nlam = 0;
  SegHost S;
  int64_t nrows = 0, npad = 0;
  // stacked operator (device)
  DevBuf sptr, scol, K, M, E, bidx, diag, Bb, A, A32, d, dinv;
  // split form of the stacked operator (no absorption field; HZ_SPLIT=0
  // turns it off): real parts, int16 column offsets when they fit, and the
  // interleaved lists of the entries that carry a wall or interface term or
  // sit in such a node's column (their 1 / diag is complex)
  bool split = false, dcol16 = false;
  int64_t n_islots = 0;
  DevBuf dcol, imeta, icol, ipos, R, R32, I, I32;
  std::vector<double> bmass;         // [nbe][NTAG] host
  bool eta = false;
  // interface maps (device)
  DevBuf rowS, rowT, sw, mptr, mcol, mval;
  DevBuf srow, sptr2, sidx;          // scatter of multipliers to stacked rows
  int64_t nsrow = 0;
  DevBuf g2r_ptr, g2r_row;           // glue: stacked rows of every global node
  DevBuf l2g, winv;                  // stacked row -> global node, 1 / multiplicity
  double alpha_k = -1.0;             // k and coefficients the operator was formed for
  std::complex<double> alpha_lo, alpha_hi;
};

template <typename V>
int up(hz_ctx ctx, DevBuf& b, const std::vector<V>& h) {
  size_t before = b.bytes;
  HZ_TRY(b.ensure(sizeof(V) * std::max<size_t>(h.size(), 1)));
  ctx->dev_bytes += int64_t(b.bytes) - int64_t(before);
  if (!h.empty()) HZ_HIP(hipMemcpy(b.p, h.data(), sizeof(V) * h.size(), hipMemcpyHostToDevice));
  return HZ_OK;
}

inline int64_t gid(int64_t i, int64_t j, int64_t k, int64_t nx, int64_t ny) { return i + (nx + 1) * (j + (ny + 1) * k); }

int check_structured(hz_ctx ctx) {
  const HostAsm& a = ctx->h;
  const int64_t nx = ctx->elems[0], ny = ctx->elems[1], nz = ctx->elems[2];
  if (nx < 1 || ny < 1 || nz < 1) return hz_fail(HZ_ERR_INVALID, "Schwarz needs mesh->elems of a structured box");
  if (!ctx->perm.empty()) return hz_fail(HZ_ERR_INVALID, "Schwarz needs the mesh's own node numbering");
  if (a.npe != 8) return hz_fail(HZ_ERR_INVALID, "Schwarz needs a hexahedral mesh");
  if (int64_t(a.n) != (nx + 1) * (ny + 1) * (nz + 1) || int64_t(a.ne) != nx * ny * nz)
    return hz_fail(HZ_ERR_INVALID, "Schwarz: node/element counts do not match elems");
  for (int d = 0; d < 3; ++d)
    if (ctx->parts[d] < 1 || ctx->parts[d] > ctx->elems[d])
      return hz_fail(HZ_ERR_INVALID, "Schwarz: parts[%d]=%d not in 1..%d", d, ctx->parts[d], ctx->elems[d]);
  for (int64_t e = 0; e < a.ne; ++e) {
    int64_t ei = e % nx, ej = (e / nx) % ny, ek = e / (nx * ny);
    for (int l = 0; l < 8; ++l) {
      int64_t want = gid(ei + (l & 1), ej + ((l >> 1) & 1), ek + ((l >> 2) & 1), nx, ny);
      if (a.hex[e * 8 + l] != want) return hz_fail(HZ_ERR_INVALID, "Schwarz: mesh is not the structured box numbering");
    }
  }
  return HZ_OK;
}

int build_dd(hz_ctx ctx, DDData* D) {
  HZ_TRY(check_structured(ctx));
  const HostAsm& g = ctx->h;
  const int64_t nx = ctx->elems[0], ny = ctx->elems[1], nz = ctx->elems[2];
  const int64_t cnt[3] = {nx, ny, nz};
  const int px = ctx->parts[0], py = ctx->parts[1], pz = ctx->parts[2];
  for (int d = 0; d < 3; ++d) D->parts[d] = ctx->parts[d];
  D->nsub = px * py * pz;
  D->subs.resize(D->nsub);
  auto cut = [&](int d, int a) { return int((int64_t(a) * cnt[d]) / D->parts[d]); };
  // owner of every global wall face: subdomain of its adjacent element
  std::vector<std::vector<int64_t>> owned(D->nsub);
  auto part_of = [&](int d, int64_t e) {
    int a = 0;
    while (a + 1 < D->parts[d] && cut(d, a + 1) <= e) ++a;
    return a;
  };
  for (int64_t f = 0; f < g.nb; ++f) {
    int64_t mn[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
    for (int l = 0; l < 4; ++l) {
      int64_t v = g.bface[f * 4 + l];
      int64_t c3[3] = {v % (nx + 1), (v / (nx + 1)) % (ny + 1), v / ((nx + 1) * (ny + 1))};
      for (int d = 0; d < 3; ++d) mn[d] = std::min(mn[d], c3[d]);
    }
    int q[3];
    for (int d = 0; d < 3; ++d) q[d] = part_of(d, std::min(mn[d], cnt[d] - 1));
    owned[q[0] + px * (q[1] + py * q[2])].push_back(f);
  }
  std::vector<int32_t> mult(g.n, 0);
  int64_t row_off = 0;
  for (int c = 0; c < pz; ++c)
    for (int b = 0; b < py; ++b)
      for (int a = 0; a < px; ++a) {
        const int s = a + px * (b + py * c);
        DDSub& U = D->subs[s];
        const int pos[3] = {a, b, c};
        for (int d = 0; d < 3; ++d) {
          U.lo[d] = cut(d, pos[d]);
          U.ln[d] = cut(d, pos[d] + 1) - U.lo[d];
        }
        const int64_t lx = U.ln[0], ly = U.ln[1], lz = U.ln[2];
        auto lid = [&](int64_t i, int64_t j, int64_t k) { return i + (lx + 1) * (j + (ly + 1) * k); };
        U.n = (lx + 1) * (ly + 1) * (lz + 1);
        U.l2g.resize(U.n);
        std::vector<double> xyz(U.n * 3);
        for (int64_t k = 0; k <= lz; ++k)
          for (int64_t j = 0; j <= ly; ++j)
            for (int64_t i = 0; i <= lx; ++i) {
              int64_t l = lid(i, j, k), G = gid(i + U.lo[0], j + U.lo[1], k + U.lo[2], nx, ny);
              U.l2g[l] = int32_t(G);
              mult[G] += 1;
              for (int d = 0; d < 3; ++d) xyz[l * 3 + d] = g.xyz[G * 3 + d];
            }
        std::vector<int32_t> hex(lx * ly * lz * 8);
        std::vector<double> eta;   // the subdomain's share of the loss field
        if (!g.Meta.empty() && !ctx->eta_field.empty()) eta.resize(lx * ly * lz);
        for (int64_t k = 0; k < lz; ++k)
          for (int64_t j = 0; j < ly; ++j)
            for (int64_t i = 0; i < lx; ++i) {
              int64_t e = i + lx * (j + ly * k);
              for (int l = 0; l < 8; ++l) hex[e * 8 + l] = int32_t(lid(i + (l & 1), j + ((l >> 1) & 1), k + ((l >> 2) & 1)));
            }
        std::vector<int32_t> bf, tag;
        std::vector<uint8_t> src;
        for (int64_t f : owned[s]) {
          for (int l = 0; l < 4; ++l) {
            int64_t v = g.bface[f * 4 + l];
            int64_t gi = v % (nx + 1), gj = (v / (nx + 1)) % (ny + 1), gk = v / ((nx + 1) * (ny + 1));
            bf.push_back(int32_t(lid(gi - U.lo[0], gj - U.lo[1], gk - U.lo[2])));
          }
          tag.push_back(g.btag[f]);
          src.push_back(g.bsrc[f]);
        }
        for (int d = 0; d < 3; ++d) {
          int a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;
          for (int side = 0; side < 2; ++side) {
            int plane = side ? U.lo[d] + U.ln[d] : U.lo[d];
            if (plane == 0 || plane == cnt[d]) continue;
            for (int64_t v = 0; v < U.ln[a2]; ++v)
              for (int64_t u = 0; u < U.ln[a1]; ++u) {
                for (int bb = 0; bb < 2; ++bb)
                  for (int aa = 0; aa < 2; ++aa) {
                    int64_t idx[3];
                    idx[d] = side * U.ln[d];
                    idx[a1] = u + aa;
                    idx[a2] = v + bb;
                    bf.push_back(int32_t(lid(idx[0], idx[1], idx[2])));
                  }
                tag.push_back(6 + 2 * d + side);
                src.push_back(0);
              }
          }
        }
        hz_mesh m = {};
        m.n_nodes = int32_t(U.n);
        m.n_elems = int32_t(lx * ly * lz);
        m.n_bfaces = int32_t(tag.size());
        m.xyz = xyz.data();
        m.hex = hex.data();
        m.bface = bf.data();
        m.bface_tag = tag.data();
        m.bface_src = src.data();
        m.c = ctx->c;
        if (!eta.empty()) {
          for (int64_t k = 0; k < lz; ++k)
            for (int64_t j = 0; j < ly; ++j)
              for (int64_t i = 0; i < lx; ++i)
                eta[i + lx * (j + ly * k)] = ctx->eta_field[(i + U.lo[0]) + nx * ((j + U.lo[1]) + ny * (k + U.lo[2]))];
        }
        HZ_TRY(host_assemble(&m, eta.empty() ? nullptr : eta.data(), &U.a, NTAG));
        U.nrows = int64_t(ceil_div(U.n, kBlock)) * kBlock;
        U.row_off = row_off;
        row_off += U.nrows;
      }
  D->nrows = row_off;
  D->eta = !g.Meta.empty();
  // stacked sliced-ELL system
  std::vector<int32_t> sptr(1, 0), scol, bidx, dpos(row_off, -1), l2g(row_off, 0);
  std::vector<uint8_t> real_slot;   // 1 for a stored entry (0: slice padding)
  std::vector<double> K, M, E, winv(row_off, 0.0);
  D->bmass.clear();
  int64_t slot_off = 0;
  for (int s = 0; s < D->nsub; ++s) {
    DDSub& U = D->subs[s];
    SellHost sh;
    build_sell(U.a, U.nrows, &sh);
    const int64_t base = sptr.back();
    for (int32_t sl = 0; sl < sh.n_slices; ++sl) sptr.push_back(int32_t(base + sh.ptr[sl + 1]));
    std::vector<int32_t> csr2b(U.a.col.size(), -1);
    for (size_t e = 0; e < U.a.bpos.size(); ++e) csr2b[U.a.bpos[e]] = int32_t(slot_off + e);
    for (int64_t p = 0; p < sh.n_pad; ++p) {
      scol.push_back(int32_t(sh.col[p] + U.row_off));
      int64_t q = sh.src[p];
      K.push_back(q >= 0 ? U.a.K[q] : 0.0);
      M.push_back(q >= 0 ? U.a.M[q] : 0.0);
      if (D->eta) E.push_back(q >= 0 ? U.a.Meta[q] : 0.0);
      bidx.push_back(q >= 0 ? csr2b[q] : -1);
      real_slot.push_back(q >= 0 ? 1 : 0);
    }
    for (int64_t i = 0; i < U.n; ++i) {
      dpos[U.row_off + i] = int32_t(base + sh.ptr[i / kWave] + (U.a.diag[i] - U.a.rowptr[i]) * kWave + (i % kWave));
      l2g[U.row_off + i] = U.l2g[i];
      winv[U.row_off + i] = 1.0 / mult[U.l2g[i]];
    }
    D->bmass.insert(D->bmass.end(), U.a.bmass.begin(), U.a.bmass.end());
    slot_off += int64_t(U.a.bpos.size());
  }
  D->npad = sptr.back();
  if (D->npad >= (int64_t(1) << 31)) return hz_fail(HZ_ERR_INVALID, "Schwarz: stacked system too large");
  HZ_TRY(up(ctx, D->sptr, sptr));
  HZ_TRY(up(ctx, D->scol, scol));
  HZ_TRY(up(ctx, D->K, K));
  HZ_TRY(up(ctx, D->M, M));
  if (D->eta) HZ_TRY(up(ctx, D->E, E));
  HZ_TRY(up(ctx, D->bidx, bidx));
  HZ_TRY(up(ctx, D->diag, dpos));
  HZ_TRY(up(ctx, D->l2g, l2g));
  HZ_TRY(up(ctx, D->winv, winv));
  {
    // split form (the global operator's layout, section of ctx_upload)
    const char* env = std::getenv("HZ_SPLIT");
    D->split = !D->eta && !(env && env[0] == '0');
    if (D->split) {
      const int64_t nsl = row_off / kWave;
      std::vector<int16_t> dc(D->npad, 0);
      bool fits = true;
      std::vector<ImSlice> meta(nsl);
      std::vector<int32_t> pcol, ppos;
      std::vector<std::vector<std::pair<int32_t, int32_t>>> lists(kWave);   // per lane: (column, position)
      int64_t lanes = 0;
      for (int64_t sl = 0; sl < nsl; ++sl) {
        const int64_t w = (sptr[sl + 1] - sptr[sl]) / kWave;
        ImSlice m{int32_t(pcol.size()), 0, 0, int32_t(lanes), 0ull};
        for (int l = 0; l < kWave; ++l) {
          lists[l].clear();
          const int64_t r = sl * kWave + l;
          for (int64_t k = 0; k < w; ++k) {
            const int64_t p = sptr[sl] + k * kWave + l;
            if (!real_slot[p]) continue;   // padding: value 0, offset 0 (the row itself)
            const int64_t d = int64_t(scol[p]) - r;
            if (d < -32768 || d > 32767) fits = false;
            else dc[p] = int16_t(d);
            const int32_t cd = dpos[scol[p]];
            if (bidx[p] >= 0 || (cd >= 0 && bidx[cd] >= 0)) lists[l].push_back({scol[p], int32_t(p)});
          }
          if (!lists[l].empty()) {
            m.mask |= 1ull << l;
            ++m.nl;
            m.w = std::max<int32_t>(m.w, int32_t(lists[l].size()));
          }
        }
        const size_t at0 = pcol.size();
        pcol.resize(at0 + size_t(m.w) * m.nl);
        ppos.resize(at0 + size_t(m.w) * m.nl);
        int j = 0;
        for (int l = 0; l < kWave; ++l) {
          if (!((m.mask >> l) & 1ull)) continue;
          for (int k = 0; k < m.w; ++k) {
            const size_t at = at0 + size_t(k) * m.nl + j;
            const bool on = k < int(lists[l].size());
            pcol[at] = on ? lists[l][k].first : int32_t(sl * kWave + l);
            ppos[at] = on ? lists[l][k].second : -1;
          }
          ++j;
        }
        meta[sl] = m;
        lanes += m.nl;
      }
      if (pcol.size() > size_t(INT32_MAX)) return hz_fail(HZ_ERR_INVALID, "Schwarz: too many imaginary entries");
      D->dcol16 = fits;
      if (fits) HZ_TRY(up(ctx, D->dcol, dc));
      HZ_TRY(up(ctx, D->imeta, meta));
      HZ_TRY(up(ctx, D->icol, pcol));
      HZ_TRY(up(ctx, D->ipos, ppos));
      D->n_islots = int64_t(pcol.size());
    }
  }
  for (DevBuf* b : {&D->A, &D->A32}) {
    size_t before = b->bytes;
    HZ_TRY(b->ensure((b == &D->A ? sizeof(z_t) : sizeof(c_t)) * D->npad));
    ctx->dev_bytes += int64_t(b->bytes) - int64_t(before);
  }
  for (DevBuf* b : {&D->d, &D->dinv}) {
    size_t before = b->bytes;
    HZ_TRY(b->ensure(sizeof(z_t) * D->nrows));
    ctx->dev_bytes += int64_t(b->bytes) - int64_t(before);
  }
  // segments = subdomains
  D->S.nseg = D->nsub;
  D->S.nrows = D->nrows;
  D->S.nblk = int(D->nrows / kBlock);
  D->S.seg_blk.assign(1, 0);
  D->S.seg_n.clear();
  for (int s = 0; s < D->nsub; ++s) {
    D->S.seg_blk.push_back(int((D->subs[s].row_off + D->subs[s].nrows) / kBlock));
    D->S.seg_n.push_back(D->subs[s].n);
  }
  HZ_TRY(seg_upload(ctx, &D->S, "dd"));

  // interface pairs
  D->pairs.clear();
  for (int c = 0; c < pz; ++c)
    for (int b = 0; b < py; ++b)
      for (int a = 0; a < px; ++a) {
        const int s = a + px * (b + py * c);
        const int pos[3] = {a, b, c};
        for (int d = 0; d < 3; ++d)
          for (int side = 0; side < 2; ++side) {
            int q[3] = {pos[0], pos[1], pos[2]};
            q[d] += side ? 1 : -1;
            if (q[d] < 0 || q[d] >= D->parts[d]) continue;
            DDPair P;
            P.s = s;
            P.t = q[0] + px * (q[1] + py * q[2]);
            P.tag = 6 + 2 * d + side;
            const HostAsm& as = D->subs[s].a;
            std::vector<int32_t> gl;
            for (int64_t f = 0; f < as.nb; ++f)
              if (as.btag[f] == P.tag)
                for (int l = 0; l < 4; ++l) gl.push_back(D->subs[s].l2g[as.bface[f * 4 + l]]);
            std::sort(gl.begin(), gl.end());
            gl.erase(std::unique(gl.begin(), gl.end()), gl.end());
            P.g = gl;
            std::map<int32_t, int32_t> pos_of;
            for (size_t i = 0; i < gl.size(); ++i) pos_of[gl[i]] = int32_t(i);
            // local ids in s and t
            auto local_of = [&](const DDSub& U, int32_t G) {
              int64_t gi = G % (nx + 1), gj = (G / (nx + 1)) % (ny + 1), gk = G / ((nx + 1) * (ny + 1));
              return int32_t((gi - U.lo[0]) + (U.ln[0] + 1) * ((gj - U.lo[1]) + (U.ln[1] + 1) * (gk - U.lo[2])));
            };
            for (int32_t G : gl) {
              P.ins.push_back(local_of(D->subs[s], G));
              P.int_.push_back(local_of(D->subs[P.t], G));
            }
            // interface-face mass over G (faces in order: fixed summation order)
            std::map<std::pair<int32_t, int32_t>, double> ent;
            for (int64_t f = 0; f < as.nb; ++f) {
              if (as.btag[f] != P.tag) continue;
              double X[4][3], Fe[4][4];
              int32_t pn[4];
              for (int l = 0; l < 4; ++l) {
                int32_t v = as.bface[f * 4 + l];
                pn[l] = pos_of[D->subs[s].l2g[v]];
                for (int dd = 0; dd < 3; ++dd) X[l][dd] = as.xyz[int64_t(v) * 3 + dd];
              }
              q1::quad_mass(X, Fe);
              for (int l = 0; l < 4; ++l)
                for (int o = 0; o < 4; ++o) ent[{pn[l], pn[o]}] += Fe[l][o];
            }
            P.mptr.assign(gl.size() + 1, 0);
            for (auto& kv : ent) P.mptr[kv.first.first + 1]++;
            for (size_t i = 0; i < gl.size(); ++i) P.mptr[i + 1] += P.mptr[i];
            for (auto& kv : ent) {
              P.mcol.push_back(kv.first.second);
              P.mval.push_back(kv.second);
            }
            D->pairs.push_back(std::move(P));
          }
      }
  std::map<std::pair<int, int>, int> idx;
  D->lam_off.assign(1, 0);
  for (size_t i = 0; i < D->pairs.size(); ++i) {
    idx[{D->pairs[i].s, D->pairs[i].t}] = int(i);
    D->lam_off.push_back(D->lam_off.back() + int64_t(D->pairs[i].g.size()));
  }
  D->nlam = D->lam_off.back();
  std::vector<int32_t> rowS(D->nlam), rowT(D->nlam), sw(D->nlam), mptr(1, 0), mcol;
  std::vector<double> mval;
  for (size_t i = 0; i < D->pairs.size(); ++i) {
    const DDPair& P = D->pairs[i];
    const int j = idx[{P.t, P.s}];
    if (D->pairs[j].g != P.g) return hz_fail(HZ_ERR_INVALID, "Schwarz: interface node sets differ");
    const int64_t o = D->lam_off[i];
    for (size_t q = 0; q < P.g.size(); ++q) {
      rowS[o + q] = int32_t(D->subs[P.s].row_off + P.ins[q]);
      rowT[o + q] = int32_t(D->subs[P.t].row_off + P.int_[q]);
      sw[o + q] = int32_t(D->lam_off[j] + q);
      for (int32_t e = P.mptr[q]; e < P.mptr[q + 1]; ++e) {
        mcol.push_back(int32_t(o + P.mcol[e]));
        mval.push_back(P.mval[e]);
      }
      mptr.push_back(int32_t(mcol.size()));
    }
  }
  HZ_TRY(up(ctx, D->rowS, rowS));
  HZ_TRY(up(ctx, D->rowT, rowT));
  HZ_TRY(up(ctx, D->sw, sw));
  HZ_TRY(up(ctx, D->mptr, mptr));
  HZ_TRY(up(ctx, D->mcol, mcol));
  HZ_TRY(up(ctx, D->mval, mval));
  // scatter lists: for every stacked interface row, its multiplier entries (ascending)
  std::vector<std::pair<int32_t, int32_t>> rs;
  for (int64_t q = 0; q < D->nlam; ++q) rs.push_back({rowS[q], int32_t(q)});
  std::sort(rs.begin(), rs.end());
  std::vector<int32_t> srow, sp(1, 0), sidx;
  for (size_t q = 0; q < rs.size(); ++q) {
    if (srow.empty() || srow.back() != rs[q].first) {
      if (!srow.empty()) sp.push_back(int32_t(sidx.size()));
      srow.push_back(rs[q].first);
    }
    sidx.push_back(rs[q].second);
  }
  if (!srow.empty()) sp.push_back(int32_t(sidx.size()));
  D->nsrow = int64_t(srow.size());
  HZ_TRY(up(ctx, D->srow, srow));
  HZ_TRY(up(ctx, D->sptr2, sp));
  HZ_TRY(up(ctx, D->sidx, sidx));
  // glue lists: stacked rows of every global node, in subdomain order
  std::vector<int32_t> gp(g.n + 1, 0), gr;
  for (int64_t r = 0; r < row_off; ++r)
    if (winv[r] > 0) gp[l2g[r] + 1]++;
  for (int64_t i = 0; i < g.n; ++i) gp[i + 1] += gp[i];
  gr.assign(gp[g.n], 0);
  {
    std::vector<int32_t> fill(gp.begin(), gp.end() - 1);
    for (int64_t r = 0; r < row_off; ++r)
      if (winv[r] > 0) gr[fill[l2g[r]]++] = int32_t(r);
  }
  HZ_TRY(up(ctx, D->g2r_ptr, gp));
  HZ_TRY(up(ctx, D->g2r_row, gr));
  return HZ_OK;
}

// A Robin coefficient alpha enters as an interface "admittance" alpha / (i k):
// the operator forming adds i k beta_tag M_tag for every boundary tag.  Tag
// 6 + 2d + side is the interface face on the low (side 0) or high (side 1)
// end of axis d: on a high face the subdomain is the lower-index side (a_lo).
int form_dd_operator(hz_ctx ctx, DDData* D, std::complex<double> a_lo, std::complex<double> a_hi,
                     bool want32) {
  const double k = ctx->k;
  const std::complex<double> ik(0.0, k);
  const std::complex<double> b_lo = (k > 0.0) ? a_lo / ik : 0.0, b_hi = (k > 0.0) ? a_hi / ik : 0.0;
  const int64_t nbe = int64_t(D->bmass.size()) / NTAG;
  std::vector<z_t> Bb(std::max<int64_t>(nbe, 1), z_t{0.0, 0.0});
  for (int64_t e = 0; e < nbe; ++e) {
    std::complex<double> acc = 0.0;
    for (int w = 0; w < 6; ++w) acc += ctx->beta[w] * D->bmass[e * NTAG + w];
    for (int w = 6; w < NTAG; ++w) acc += ((w - 6) % 2 == 1 ? b_lo : b_hi) * D->bmass[e * NTAG + w];
    Bb[e] = z_t{acc.real(), acc.imag()};
  }
  HZ_TRY(up(ctx, D->Bb, Bb));
  OpParts P;
  P.K = D->K.as<double>();
  P.M = D->M.as<double>();
  P.Meta = D->eta ? D->E.as<double>() : nullptr;
  P.bidx = D->bidx.as<int>();
  P.Bb = D->Bb.as<z_t>();
  P.diag = D->diag.as<int>();
  if (D->split) {
    HZ_TRY(D->R.ensure(sizeof(double) * D->npad));
    HZ_TRY(D->I.ensure(sizeof(double) * std::max<int64_t>(D->n_islots, 1)));
    if (want32) {
      HZ_TRY(D->R32.ensure(sizeof(float) * D->npad));
      HZ_TRY(D->I32.ensure(sizeof(float) * std::max<int64_t>(D->n_islots, 1)));
    }
  }
  HZ_TRY(op_form(ctx->stream, D->nrows, D->nrows, D->npad, D->scol.as<int>(), P, k, 1, D->A.as<z_t>(),
                 want32 ? D->A32.as<c_t>() : nullptr, D->d.as<z_t>(), D->dinv.as<z_t>(),
                 D->split ? D->R.as<double>() : nullptr, D->split && want32 ? D->R32.as<float>() : nullptr));
  if (D->split)
    HZ_TRY(op_split_im(ctx->stream, D->n_islots, D->ipos.as<int>(), D->A.as<z_t>(), D->I.as<double>(),
                       want32 ? D->I32.as<float>() : nullptr));
  D->alpha_k = k;
  D->alpha_lo = a_lo;
  D->alpha_hi = a_hi;
  return HZ_OK;
}

// ---------------------------------------------------------------- interface kernels
// rhs[row] = base[row] (or 0) for all stacked rows
__global__ void k_dd_split(int64_t nrows, const z_t* __restrict__ f, const int* __restrict__ l2g,
                           const double* __restrict__ winv, z_t* __restrict__ rhs) {
  int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (r >= nrows) return;
  double w = winv[r];
  rhs[r] = w > 0.0 ? w * f[l2g[r]] : z_t{0.0, 0.0};
}

// rhs[srow[i]] += sum of the multipliers scattered to that row (fixed order)
__global__ void k_dd_scatter(int64_t nsrow, const int* __restrict__ srow, const int* __restrict__ sptr,
                             const int* __restrict__ sidx, const z_t* __restrict__ lam, z_t* __restrict__ rhs) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= nsrow) return;
  z_t acc = rhs[srow[i]];
  for (int q = sptr[i]; q < sptr[i + 1]; ++q) acc = acc + lam[sidx[q]];
  rhs[srow[i]] = acc;
}

// u = dinv .* uhat (stacked)
__global__ void k_dd_unscale(int64_t nrows, const z_t* __restrict__ dinv, z_t* __restrict__ u) {
  int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (r < nrows) u[r] = dinv[r] * u[r];
}

// y = s_lam * lam + s_sw * lam[sw] + s_t * (a_lo + a_hi) M_G R_ts u
__global__ void k_dd_update(int64_t nlam, const z_t* __restrict__ lam, const int* __restrict__ sw,
                            const int* __restrict__ mptr, const int* __restrict__ mcol, const double* __restrict__ mval,
                            const int* __restrict__ rowT, const z_t* __restrict__ u, z_t two_alpha, double s_lam,
                            double s_sw, double s_t, z_t* __restrict__ y) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= nlam) return;
  z_t m = {0.0, 0.0};
  for (int q = mptr[i]; q < mptr[i + 1]; ++q) {
    z_t v = u[rowT[mcol[q]]];
    m.re = fma(mval[q], v.re, m.re);
    m.im = fma(mval[q], v.im, m.im);
  }
  z_t t = two_alpha * m;
  z_t r = {0.0, 0.0};
  if (s_lam != 0.0) r = s_lam * lam[i];
  if (s_sw != 0.0) r = r + s_sw * lam[sw[i]];
  y[i] = r + s_t * t;
}

// p[g] = mean of u over the stacked rows of global node g
__global__ void k_dd_glue(int64_t n, const int* __restrict__ gp, const int* __restrict__ gr, const z_t* __restrict__ u,
                          z_t* __restrict__ p) {
  int64_t g = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (g >= n) return;
  z_t acc = {0.0, 0.0};
  int q0 = gp[g], q1 = gp[g + 1];
  for (int q = q0; q < q1; ++q) acc = acc + u[gr[q]];
  double w = 1.0 / double(q1 - q0);
  p[g] = w * acc;
}

__global__ void k_axpy_z(int64_t n, z_t a, const z_t* __restrict__ x, z_t* __restrict__ y) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) y[i] = y[i] + a * x[i];
}

__global__ void k_scal_z(int64_t n, z_t a, const z_t* __restrict__ x, z_t* __restrict__ y) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// ---------------------------------------------------------------- driver
struct DDRun {
  hz_ctx ctx;
  DDData* D;
  hz_solve_opts lo;        // local solve options
  bool mixed;
  z_t *rhs, *u, *tmp;      // stacked vectors
  int64_t local_mv = 0;
  int nlocal = 0;

  int local_solve(const z_t* f_stacked_or_null, const z_t* lam) {
    hipStream_t s = ctx->stream;
    const int64_t nr = D->nrows;
    if (f_stacked_or_null) {
      HZ_HIP(hipMemcpyAsync(rhs, f_stacked_or_null, sizeof(z_t) * nr, hipMemcpyDeviceToDevice, s));
    } else {
      HZ_TRY(op_fill(s, nr, rhs, z_t{0.0, 0.0}));
    }
    if (lam && D->nsrow > 0) {
      k_dd_scatter<<<ceil_div(D->nsrow, kBlock), kBlock, 0, s>>>(D->nsrow, D->srow.as<int>(), D->sptr2.as<int>(),
                                                              D->sidx.as<int>(), lam, rhs);
      HZ_HIP(hipGetLastError());
    }
    HZ_TRY(op_fill(s, nr, u, z_t{0.0, 0.0}));
    // the split form when formed (no absorption field), else complex values
    auto split_op = [&](auto* re, auto* im, auto& A) {
      A.dcol = D->dcol16 ? D->dcol.as<int16_t>() : nullptr;
      A.imeta = D->imeta.as<ImSlice>();
      A.icol = D->icol.as<int>();
      A.re = re;
      A.iim = im;
    };
    SellOp<double> A64;
    A64.ptr = D->sptr.as<int>();
    A64.col = D->scol.as<int>();
    if (D->split) split_op(D->R.as<double>(), D->I.as<double>(), A64);
    else A64.val = D->A.as<z_t>();
    if (mixed) {
      SellOp<float> A32;
      A32.ptr = A64.ptr;
      A32.col = A64.col;
      if (D->split) split_op(D->R32.as<float>(), D->I32.as<float>(), A32);
      else A32.val = D->A32.as<c_t>();
      IrOut io;
      HZ_TRY(ir_run(ctx, D->S, A64, A32, rhs, u, lo, &io, "dd"));
      local_mv += io.matvecs + io.inner_matvecs;
    } else {
      KrylovCtl c;
      c.tol = lo.tol;
      c.max_matvec = lo.max_matvec;
      c.restart = lo.restart;
      c.ell = lo.restart;
      KrylovOut ko;
      HZ_TRY(krylov_run<double>(ctx, lo.method, D->S, A64, rhs, u, c, &ko, "dd"));
      int mx = 0;
      for (int m : ko.matvecs) mx = std::max(mx, m);
      local_mv += mx;
    }
    nlocal += 1;
    k_dd_unscale<<<ceil_div(nr, kBlock), kBlock, 0, s>>>(nr, D->dinv.as<z_t>(), u);
    HZ_HIP(hipGetLastError());
    return HZ_OK;
  }

  // y = (I - B) lam  (homogeneous), or c = B(0) with f when f != NULL
  int apply(const z_t* lam, z_t* y, const z_t* f_st) {
    HZ_TRY(local_solve(f_st, lam));
    const std::complex<double> sum = D->alpha_lo + D->alpha_hi;   // T_st + T_ts
    z_t ta = {sum.real(), sum.imag()};
    const int64_t nl = D->nlam;
    if (f_st) {   // c = (a_lo + a_hi) M_G R u(f)
      k_dd_update<<<ceil_div(nl, kBlock), kBlock, 0, ctx->stream>>>(nl, y, D->sw.as<int>(), D->mptr.as<int>(),
          D->mcol.as<int>(), D->mval.as<double>(), D->rowT.as<int>(), u, ta, 0.0, 0.0, 1.0, y);
    } else {      // (I - B) lam = lam + lam_sw - (a_lo + a_hi) M_G R u(lam)
      k_dd_update<<<ceil_div(nl, kBlock), kBlock, 0, ctx->stream>>>(nl, lam, D->sw.as<int>(), D->mptr.as<int>(),
          D->mcol.as<int>(), D->mval.as<double>(), D->rowT.as<int>(), u, ta, 1.0, 1.0, -1.0, y);
    }
    HZ_HIP(hipGetLastError());
    return HZ_OK;
  }
};

}  // namespace

// Optimised Robin coefficients (p + i q with p, q > 0) for the half-space
// model of an interface: the interface modes xi resolvable between the
// subdomain width H and the mesh spacing h, xi in [pi/H, pi/h], have the
// transparent-condition symbol l(xi) = sqrt(xi^2 - k^2) (evanescent) or
// i sqrt(k^2 - xi^2) (propagating, e^{+i w t} convention); the modes within
// pi/(2H) of k, where every factor tends to one, are left out.
//   one-sided: alpha minimises max |(l - alpha) / (l + alpha)| over a log
//     grid of 80 x 80 (p, q);
//   two-sided: (a_lo, a_hi) = (p_lo + i q, p_hi + i q) with q of the
//     one-sided optimum; (p_lo, p_hi) minimise the factor of a double step,
//     max |(l - a_lo)(l - a_hi) / ((l + a_lo)(l + a_hi))|, by a pattern search
//     in log(p) started from the one-sided p split apart by factors 1 .. 16
//     (the best start wins).  Keeping q keeps the local problems absorbing:
//     the model's modes are all evanescent when k < pi/H, and a real pair
//     (which the model would prefer) leaves the subdomains of a nearly
//     lossless cavity without damping, which slows their inexact solves.
void dd_optimised_alpha(double k, double Hsub, double h, int sides, std::complex<double>* out) {
  const double xmin = M_PI / Hsub, xmax = M_PI / h;
  std::vector<std::complex<double>> lam;
  const int nx = 2000;
  for (int i = 0; i < nx; ++i) {
    double xi = xmin * std::pow(xmax / xmin, double(i) / (nx - 1));
    if (std::fabs(xi - k) <= 0.5 * xmin) continue;
    lam.push_back(xi > k ? std::complex<double>(std::sqrt(xi * xi - k * k), 0.0)
                         : std::complex<double>(0.0, std::sqrt(k * k - xi * xi)));
  }
  const int ng = 80;
  double lo = xmin / 10.0, best = 1e300;
  std::complex<double> arg(0.0, k);
  for (int ip = 0; ip < ng; ++ip) {
    double pv = lo * std::pow(xmax / lo, double(ip) / (ng - 1));
    for (int iq = 0; iq < ng; ++iq) {
      double qv = lo * std::pow(xmax / lo, double(iq) / (ng - 1));
      std::complex<double> a(pv, qv);
      double worst = 0.0;
      for (const auto& l : lam) worst = std::max(worst, std::abs((l - a) / (l + a)));
      if (worst < best) {
        best = worst;
        arg = a;
      }
    }
  }
  out[0] = out[1] = arg;
  if (sides != 2 || lam.empty()) return;
  const double q = arg.imag();
  auto factor = [&](const double* v) {   // v = log p_lo, log p_hi
    const std::complex<double> a1(std::exp(v[0]), q), a2(std::exp(v[1]), q);
    double worst = 0.0;
    for (const auto& l : lam) worst = std::max(worst, std::abs((l - a1) * (l - a2) / ((l + a1) * (l + a2))));
    return worst;
  };
  double bestv[2] = {std::log(arg.real()), std::log(arg.real())};
  double bestf = factor(bestv);
  for (double split : {1.0, 2.0, 4.0, 8.0, 16.0}) {
    double v[2] = {std::log(arg.real() / split), std::log(arg.real() * split)};
    double fv = factor(v);
    for (double step = std::log(2.0); step > 1e-3;) {
      bool moved = false;
      for (int c = 0; c < 2; ++c)
        for (double sg : {1.0, -1.0}) {
          double t[2] = {v[0], v[1]};
          t[c] += sg * step;
          const double ft = factor(t);
          if (ft < fv) {
            fv = ft;
            v[0] = t[0];
            v[1] = t[1];
            moved = true;
          }
        }
      if (!moved) step *= 0.5;
    }
    if (fv < bestf) {
      bestf = fv;
      bestv[0] = v[0];
      bestv[1] = v[1];
    }
  }
  out[0] = std::complex<double>(std::exp(bestv[0]), q);
  out[1] = std::complex<double>(std::exp(bestv[1]), q);
}

namespace {

int host_dot(hz_ctx ctx, int64_t n, const z_t* a, const z_t* b, std::complex<double>* out) {
  int rc = 0;
  DevBuf* r = ctx->buf("dd.dot", 16, &rc);
  if (rc) return rc;
  HZ_TRY(op_dotc(ctx, n, a, b, r->as<double>()));
  double h[2];
  HZ_HIP(hipMemcpyAsync(h, r->p, 16, hipMemcpyDeviceToHost, ctx->stream));
  HZ_HIP(hipStreamSynchronize(ctx->stream));
  *out = std::complex<double>(h[0], h[1]);
  return HZ_OK;
}

}  // namespace

int schwarz_solve(hz_ctx ctx, const hz_solve_opts& o, const z_t* f, z_t* p, hz_solve_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  if (!ctx->dd_data || ctx->dd_version != ctx->params_version) {
    ctx->dd_data.reset();
    std::shared_ptr<void> d(new DDData(), [](void* q) { delete static_cast<DDData*>(q); });
    HZ_TRY(build_dd(ctx, static_cast<DDData*>(d.get())));
    ctx->dd_data = d;
    ctx->dd_version = ctx->params_version;
  }
  DDData* D = static_cast<DDData*>(ctx->dd_data.get());
  const bool mixed = o.precision == HZ_MIXED;
  std::complex<double> alpha(o.dd_alpha.re, o.dd_alpha.im), alpha2(o.dd_alpha2.re, o.dd_alpha2.im);
  if (alpha == 0.0) {
    double Hsub = 1e300, h = 1e300;
    const HostAsm& g = ctx->h;
    for (int d = 0; d < 3; ++d) {
      // spacing of the structured box along axis d (node 0 to its neighbour)
      int64_t step = d == 0 ? 1 : (d == 1 ? (ctx->elems[0] + 1) : int64_t(ctx->elems[0] + 1) * (ctx->elems[1] + 1));
      double hd = std::fabs(g.xyz[step * 3 + d] - g.xyz[d]);
      h = std::min(h, hd);
      for (const DDSub& U : D->subs) Hsub = std::min(Hsub, hd * U.ln[d]);
    }
    std::complex<double> opt[2] = {1.0, 1.0};
    if (ctx->k > 0.0) dd_optimised_alpha(ctx->k, Hsub, h, 2, opt);
    alpha = opt[0];
    alpha2 = opt[1];
  } else if (alpha2 == 0.0) {
    alpha2 = alpha;                    // one-sided
  }
  if (!std::isfinite(alpha.real()) || !std::isfinite(alpha.imag()) || !std::isfinite(alpha2.real()) ||
      !std::isfinite(alpha2.imag()))
    return hz_fail(HZ_ERR_INVALID, "bad dd_alpha");
  HZ_TRY(form_dd_operator(ctx, D, alpha, alpha2, mixed));
  HZ_TRY(ensure_operator(ctx, HZ_JACOBI, false));   // global operator for the final residual
  int rc = 0;
  const int64_t nr = D->nrows, nl = D->nlam, n = ctx->h.n;
  auto buf = [&](const char* nm, size_t bytes) -> z_t* {
    DevBuf* b = ctx->buf(std::string("ddv.") + nm, bytes, &rc);
    return rc ? nullptr : b->as<z_t>();
  };
  z_t* fst = buf("fst", sizeof(z_t) * nr);
  z_t* rhs = buf("rhs", sizeof(z_t) * nr);
  z_t* u = buf("u", sizeof(z_t) * nr);
  z_t* c = buf("c", sizeof(z_t) * std::max<int64_t>(nl, 1));
  z_t* lam = buf("lam", sizeof(z_t) * std::max<int64_t>(nl, 1));
  z_t* w = buf("w", sizeof(z_t) * std::max<int64_t>(nl, 1));
  const int m = o.restart;
  z_t* V = buf("V", sizeof(z_t) * std::max<int64_t>(nl, 1) * (m + 1));
  z_t* fz = buf("fz", sizeof(z_t) * ctx->sell.n_rows);
  z_t* uz = buf("uz", sizeof(z_t) * ctx->sell.n_rows);
  if (rc) return rc;
  hipStream_t s = ctx->stream;
  DDRun R;
  R.ctx = ctx;
  R.D = D;
  R.mixed = mixed;
  R.rhs = rhs;
  R.u = u;
  R.lo = o;
  R.lo.method = o.dd_inner;
  R.lo.tol = o.inner_tol > 0 ? o.inner_tol : 1e-12;   // local solves
  R.lo.inner_tol = 1e-4;                              // complex64 stage of the refinement
  R.lo.max_matvec = 100000;
  // local GMRES restart, or l of local BiCGStab(l)
  if (o.dd_inner == HZ_BICGSTABL) R.lo.restart = o.inner_restart > 0 ? o.inner_restart : 4;
  else R.lo.restart = o.inner_restart > 0 ? o.inner_restart : 30;
  // f split into subdomain shares; global f norm
  k_dd_split<<<ceil_div(nr, kBlock), kBlock, 0, s>>>(nr, f, D->l2g.as<int>(), D->winv.as<double>(), fst);
  HZ_HIP(hipGetLastError());
  SegHost* G1 = nullptr;
  HZ_TRY(ctx_single_seg(ctx, &G1));
  HZ_TRY(pad_in(ctx, n, ctx->sell.n_rows, f, nullptr, fz));
  std::vector<double> fn2;
  HZ_TRY(seg_norm2_t<double>(ctx, *G1, fz, &fn2));
  if (!std::isfinite(fn2[0])) return hz_fail(HZ_ERR_INVALID, "right-hand side has NaN/Inf entries");
  const double fnorm = std::sqrt(fn2[0]);
  hz_solve_info inf = {};
  if (fnorm == 0.0) {
    HZ_TRY(op_fill(s, n, p, z_t{0.0, 0.0}));
    HZ_HIP(hipStreamSynchronize(s));
    if (info) *info = inf;
    return HZ_OK;
  }
  int64_t if_mv = 0;
  auto glue_and_residual = [&](double* rel) -> int {
    HZ_TRY(R.local_solve(fst, nl > 0 ? lam : nullptr));
    k_dd_glue<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, D->g2r_ptr.as<int>(), D->g2r_row.as<int>(), u, p);
    HZ_HIP(hipGetLastError());
    HZ_TRY(pad_in(ctx, n, ctx->sell.n_rows, p, ctx->d_d.as<z_t>(), uz));
    std::vector<double> rr;
    HZ_TRY(true_residual(ctx, *G1, op_A(ctx), fz, uz, nullptr, &rr));
    inf.matvecs += 1;
    *rel = std::sqrt(rr[0]) / fnorm;
    return HZ_OK;
  };
  double rel = 1.0;
  if (nl == 0) {
    HZ_TRY(glue_and_residual(&rel));
  } else {
    HZ_TRY(op_fill(s, nl, lam, z_t{0.0, 0.0}));
    HZ_TRY(R.apply(nullptr, c, fst));        // c = B(0) with the load
    const int rich = o.dd_richardson;            // > 0: plain Schwarz iterations
    if (rich > 0) {
      for (int it = 0; it < rich; ++it) {
        // lam <- B lam + c = c + (a_lo + a_hi) M R u(lam) - lam_sw   ==   c - ((I - B) lam - lam)
        HZ_TRY(R.apply(lam, w, nullptr));
        k_axpy_z<<<ceil_div(nl, kBlock), kBlock, 0, s>>>(nl, z_t{-1.0, 0.0}, w, lam);   // lam - (I-B) lam
        k_axpy_z<<<ceil_div(nl, kBlock), kBlock, 0, s>>>(nl, z_t{1.0, 0.0}, c, lam);
        HZ_HIP(hipGetLastError());
        inf.iters += 1;
        if_mv += 1;
      }
      HZ_TRY(glue_and_residual(&rel));
    } else {
      // restarted GMRES on (I - B) lam = c, MGS Arnoldi with host Hessenberg
      std::complex<double> cc;
      HZ_TRY(host_dot(ctx, nl, c, c, &cc));
      const double cnorm = std::sqrt(cc.real());
      double tol_if = std::max(o.tol * 0.1, 1e-14);
      while (true) {
        bool cyc_conv = false;
        for (;;) {
          // r = c - (I - B) lam
          HZ_TRY(R.apply(lam, w, nullptr));
          if_mv += 1;
          HZ_HIP(hipMemcpyAsync(V, c, sizeof(z_t) * nl, hipMemcpyDeviceToDevice, s));
          k_axpy_z<<<ceil_div(nl, kBlock), kBlock, 0, s>>>(nl, z_t{-1.0, 0.0}, w, V);
          std::complex<double> rr;
          HZ_TRY(host_dot(ctx, nl, V, V, &rr));
          double beta = std::sqrt(rr.real());
          inf.relres_est = beta / cnorm;
          if (beta <= tol_if * cnorm) {
            cyc_conv = true;
            break;
          }
          if (if_mv + inf.matvecs >= o.max_matvec) break;
          k_scal_z<<<ceil_div(nl, kBlock), kBlock, 0, s>>>(nl, z_t{1.0 / beta, 0.0}, V, V);
          std::vector<std::complex<double>> H((m + 1) * m, 0.0), sn(m, 0.0), gv(m + 1, 0.0);
          std::vector<double> cs(m, 0.0);
          gv[0] = beta;
          int kk = 0;
          for (int j = 0; j < m; ++j) {
            z_t* vj1 = V + int64_t(j + 1) * nl;
            HZ_TRY(R.apply(V + int64_t(j) * nl, vj1, nullptr));
            if_mv += 1;
            inf.iters += 1;
            for (int i = 0; i <= j; ++i) {
              std::complex<double> h;
              HZ_TRY(host_dot(ctx, nl, V + int64_t(i) * nl, vj1, &h));
              H[i + (m + 1) * j] = h;
              k_axpy_z<<<ceil_div(nl, kBlock), kBlock, 0, s>>>(nl, z_t{-h.real(), -h.imag()}, V + int64_t(i) * nl, vj1);
            }
            std::complex<double> hh;
            HZ_TRY(host_dot(ctx, nl, vj1, vj1, &hh));
            double hn = std::sqrt(hh.real());
            H[j + 1 + (m + 1) * j] = hn;
            for (int i = 0; i < j; ++i) {
              std::complex<double> a = H[i + (m + 1) * j], b = H[i + 1 + (m + 1) * j];
              H[i + (m + 1) * j] = cs[i] * a + sn[i] * b;
              H[i + 1 + (m + 1) * j] = -std::conj(sn[i]) * a + cs[i] * b;
            }
            std::complex<double> a = H[j + (m + 1) * j], b = H[j + 1 + (m + 1) * j];
            double rho = std::sqrt(std::norm(a) + std::norm(b));
            if (rho == 0.0) {
              cs[j] = 1.0;
              sn[j] = 0.0;
            } else if (std::abs(a) == 0.0) {
              cs[j] = 0.0;
              sn[j] = 1.0;
            } else {
              cs[j] = std::abs(a) / rho;
              sn[j] = (a / std::abs(a)) * std::conj(b) / rho;
            }
            H[j + (m + 1) * j] = cs[j] * a + sn[j] * b;
            H[j + 1 + (m + 1) * j] = 0.0;
            gv[j + 1] = -std::conj(sn[j]) * gv[j];
            gv[j] = cs[j] * gv[j];
            kk = j + 1;
            double est = std::abs(gv[j + 1]);
            inf.relres_est = est / cnorm;
            if (hn == 0.0 || est <= tol_if * cnorm || if_mv + inf.matvecs >= o.max_matvec) break;
            k_scal_z<<<ceil_div(nl, kBlock), kBlock, 0, s>>>(nl, z_t{1.0 / hn, 0.0}, vj1, vj1);
            HZ_HIP(hipGetLastError());
          }
          std::vector<std::complex<double>> y(kk);
          for (int i = kk - 1; i >= 0; --i) {
            std::complex<double> acc = gv[i];
            for (int l = i + 1; l < kk; ++l) acc -= H[i + (m + 1) * l] * y[l];
            y[i] = acc / H[i + (m + 1) * i];
          }
          for (int i = 0; i < kk; ++i)
            k_axpy_z<<<ceil_div(nl, kBlock), kBlock, 0, s>>>(nl, z_t{y[i].real(), y[i].imag()}, V + int64_t(i) * nl, lam);
          HZ_HIP(hipGetLastError());
        }
        HZ_TRY(glue_and_residual(&rel));
        if (rel <= o.tol || !cyc_conv || if_mv + inf.matvecs >= o.max_matvec || tol_if <= 1e-15) break;
        tol_if *= 0.1;   // the glued residual is above tol: tighten the interface solve
      }
    }
  }
  inf.relres_true = rel;
  inf.inner_matvecs = int(std::min<int64_t>(R.local_mv, INT32_MAX));
  inf.status = (rel <= o.tol) ? HZ_OK : (std::isfinite(rel) ? HZ_NOT_CONVERGED : HZ_BREAKDOWN);
  HZ_HIP(hipStreamSynchronize(s));
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return inf.status;
}
