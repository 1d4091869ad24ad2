// Context lifecycle: device buffers, upload of the assembled operator parts
// in sliced-ELL layout, error strings.
#include <algorithm>
#include <cstdarg>
#include <cstdlib>
#include <cstring>

#include "ops.h"

namespace {
thread_local char g_err[1024] = "";
}

void hz_set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int hz_fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

const char* hz_last_error_str() { return g_err; }

int DevBuf::ensure(size_t nbytes) {
  if (nbytes <= bytes && p) return HZ_OK;
  if (p) {
    (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  if (nbytes == 0) nbytes = 16;
  hipError_t e = hipMalloc(&p, nbytes);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    return hz_fail(e == hipErrorOutOfMemory ? HZ_ERR_OOM : HZ_ERR_HIP, "hipMalloc(%zu): %s", nbytes,
                   hipGetErrorString(e));
  }
  bytes = nbytes;
  return HZ_OK;
}

DevBuf* hz_ctx_s::buf(const std::string& name, size_t nbytes, int* rc) {
  auto& slot = ws[name];
  if (!slot) slot.reset(new DevBuf());
  size_t before = slot->bytes;
  *rc = slot->ensure(nbytes);
  if (*rc) return nullptr;
  dev_bytes += int64_t(slot->bytes) - int64_t(before);
  return slot.get();
}

hz_ctx_s::~hz_ctx_s() {
  if (pinned) (void)hipHostFree(pinned);
}

int ctx_pinned(hz_ctx ctx, size_t bytes, void** out) {
  if (bytes > ctx->pinned_bytes) {
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    size_t nb = std::max<size_t>(bytes, 4096);
    HZ_HIP(hipHostMalloc(&ctx->pinned, nb, hipHostMallocDefault));
    ctx->pinned_bytes = nb;
  }
  *out = ctx->pinned;
  return HZ_OK;
}

namespace {
template <typename T>
int put(hz_ctx ctx, DevBuf& b, const T* src, size_t count) {
  size_t before = b.bytes;
  HZ_TRY(b.ensure(sizeof(T) * count));
  ctx->dev_bytes += int64_t(b.bytes) - int64_t(before);
  if (count) HZ_HIP(hipMemcpy(b.p, src, sizeof(T) * count, hipMemcpyHostToDevice));
  return HZ_OK;
}
}  // namespace

int ctx_upload_params(hz_ctx ctx) {
  const HostAsm& a = ctx->h;
  const int64_t nbe = int64_t(a.bpos.size());
  std::vector<z_t> Bb(std::max<int64_t>(nbe, 1), z_t{0.0, 0.0});
  for (int64_t e = 0; e < nbe; ++e) {
    // accumulate walls in order 0..5
    double re = 0.0, im = 0.0;
    for (int w = 0; w < 6; ++w) {
      double m = a.bmass[e * a.ntags + w];
      re += ctx->beta[w].real() * m;
      im += ctx->beta[w].imag() * m;
    }
    Bb[e] = z_t{re, im};
  }
  HZ_TRY(put(ctx, ctx->d_Bb, Bb.data(), Bb.size()));
  if (ctx->have_eta) {
    std::vector<double> v(ctx->sell.n_pad, 0.0);
    for (int64_t p = 0; p < ctx->sell.n_pad; ++p)
      if (ctx->sell.src[p] >= 0) v[p] = a.Meta[ctx->sell.src[p]];
    HZ_TRY(put(ctx, ctx->d_Meta, v.data(), v.size()));
  }
  return HZ_OK;
}

int ctx_upload(hz_ctx ctx) {
  const HostAsm& a = ctx->h;
  SellHost& s = ctx->sell;
  const int64_t nrows = int64_t(ceil_div(a.n, kBlock)) * kBlock;
  build_sell(a, nrows, &s);
  HZ_TRY(put(ctx, ctx->d_sptr, s.ptr.data(), s.ptr.size()));
  HZ_TRY(put(ctx, ctx->d_scol, s.col.data(), s.col.size()));
  {
    std::vector<double> K(s.n_pad, 0.0), M(s.n_pad, 0.0);
    for (int64_t p = 0; p < s.n_pad; ++p)
      if (s.src[p] >= 0) {
        K[p] = a.K[s.src[p]];
        M[p] = a.M[s.src[p]];
      }
    HZ_TRY(put(ctx, ctx->d_K, K.data(), K.size()));
    HZ_TRY(put(ctx, ctx->d_M, M.data(), M.size()));
  }
  {
    std::vector<int32_t> csr2b(a.col.size(), -1);
    for (size_t e = 0; e < a.bpos.size(); ++e) csr2b[a.bpos[e]] = int32_t(e);
    std::vector<int32_t> bidx(s.n_pad, -1);
    for (int64_t p = 0; p < s.n_pad; ++p)
      if (s.src[p] >= 0) bidx[p] = csr2b[s.src[p]];
    HZ_TRY(put(ctx, ctx->d_bidx, bidx.data(), bidx.size()));
  }
  std::vector<int32_t> dpos(a.n);
  for (int64_t i = 0; i < a.n; ++i)
    dpos[i] = int32_t(s.ptr[i / kWave] + (a.diag[i] - a.rowptr[i]) * kWave + (i % kWave));
  HZ_TRY(put(ctx, ctx->d_diag, dpos.data(), dpos.size()));
  {
    // Split-form pattern.  Without an absorption field, entry (i, j) of the
    // (column-scaled) operator is complex only if it carries a wall term or
    // column j's diagonal does (then 1/diag_j is complex).
    const char* env = std::getenv("HZ_SPLIT");
    ctx->split_on = !(env && env[0] == '0');
    std::vector<int32_t> csr2b(a.col.size(), -1);
    for (size_t e = 0; e < a.bpos.size(); ++e) csr2b[a.bpos[e]] = int32_t(e);
    std::vector<uint8_t> wall_col(a.n, 0);
    for (int64_t j = 0; j < a.n; ++j) wall_col[j] = csr2b[a.diag[j]] >= 0;
    std::vector<int32_t> iptr(nrows + 1, 0), icol, ipos;
    std::vector<int16_t> dcol(s.n_pad, 0);
    bool fits = true;
    for (int64_t i = 0; i < nrows; ++i) {
      if (i < a.n) {
        const int64_t sl = i / kWave, l = i % kWave, w = (s.ptr[sl + 1] - s.ptr[sl]) / kWave;
        for (int64_t k = 0; k < w; ++k) {
          const int64_t p = s.ptr[sl] + k * kWave + l;
          const int64_t d = int64_t(s.col[p]) - i;
          if (d < -32768 || d > 32767) fits = false;
          else dcol[p] = int16_t(d);
          if (s.src[p] >= 0 && (csr2b[s.src[p]] >= 0 || wall_col[s.col[p]])) {
            icol.push_back(s.col[p]);
            ipos.push_back(int32_t(p));
          }
        }
      }
      iptr[i + 1] = int32_t(icol.size());
    }
    ctx->n_imag = int64_t(icol.size());
    ctx->split_dcol = fits;
    if (fits) HZ_TRY(put(ctx, ctx->d_dcol, dcol.data(), dcol.size()));
    // interleave each slice's lists (ImSlice): entry k of the j-th listed
    // lane at base + k nl + j, shorter lists padded with position -1 (value
    // 0) and the row itself as column
    const int64_t nsl = nrows / kWave;
    std::vector<ImSlice> meta(nsl);
    std::vector<int32_t> pcol, ppos;
    for (int64_t sl = 0; sl < nsl; ++sl) {
      ImSlice m{int32_t(pcol.size()), 0, 0, 0, 0ull};
      for (int l = 0; l < kWave; ++l) {
        const int64_t r = sl * kWave + l;
        const int len = iptr[r + 1] - iptr[r];
        if (len > 0) {
          m.mask |= 1ull << l;
          ++m.nl;
          m.w = std::max(m.w, len);
        }
      }
      const size_t at0 = pcol.size();
      pcol.resize(at0 + size_t(m.w) * m.nl);
      ppos.resize(at0 + size_t(m.w) * m.nl);
      int j = 0;
      for (int l = 0; l < kWave; ++l) {
        if (!((m.mask >> l) & 1ull)) continue;
        const int64_t r = sl * kWave + l;
        for (int k = 0; k < m.w; ++k) {
          const size_t at = at0 + size_t(k) * m.nl + j;
          const int64_t q = iptr[r] + k;
          pcol[at] = q < iptr[r + 1] ? icol[q] : int32_t(r);
          ppos[at] = q < iptr[r + 1] ? ipos[q] : -1;
        }
        ++j;
      }
      meta[sl] = m;
    }
    if (pcol.size() > size_t(INT32_MAX)) return hz_fail(HZ_ERR_INVALID, "too many imaginary entries");
    ctx->n_islots = int64_t(pcol.size());
    HZ_TRY(put(ctx, ctx->d_imeta, meta.data(), meta.size()));
    HZ_TRY(put(ctx, ctx->d_icol, pcol.data(), pcol.size()));
    HZ_TRY(put(ctx, ctx->d_ipos, ppos.data(), ppos.size()));
  }
  {
    // Stencil form: a box in its own numbering stores the split values in 27
    // slots per row at the fixed neighbour offsets, without column indices.
    const char* env = std::getenv("HZ_STENCIL");
    const int64_t nx = ctx->elems[0], ny = ctx->elems[1], nz = ctx->elems[2];
    ctx->stencil_ok = false;
    if (!(env && env[0] == '0') && ctx->split_on && ctx->perm.empty() && a.npe == 8 && nx > 0 && ny > 0 &&
        nz > 0 && int64_t(a.n) == (nx + 1) * (ny + 1) * (nz + 1)) {
      StencilOffsets off;
      int t = 0;
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) off.o[t++] = int(dx + (nx + 1) * (dy + (ny + 1) * dz));
      std::vector<int32_t> src(int64_t(kStencil) * nrows, -1);
      bool ok = true;
      for (int64_t i = 0; i < a.n && ok; ++i)
        for (int64_t q = a.rowptr[i]; q < a.rowptr[i + 1]; ++q) {
          const int64_t d = int64_t(a.col[q]) - i;
          const int* k = std::lower_bound(off.o, off.o + kStencil, int(d));
          if (k == off.o + kStencil || *k != d) {
            ok = false;
            break;
          }
          src[(i / kWave) * kStencil * kWave + (k - off.o) * kWave + i % kWave] =
              int32_t(s.ptr[i / kWave] + (q - a.rowptr[i]) * kWave + i % kWave);
        }
      if (ok) {
        HZ_TRY(put(ctx, ctx->d_ssrc, src.data(), src.size()));
        ctx->soff = off;
        ctx->stencil_ok = true;
      }
    }
  }
  HZ_TRY(put(ctx, ctx->d_bmass, a.bmass.data(), a.bmass.size()));
  ctx->dirichlet = false;
  if (!a.dir.empty()) {
    // Dirichlet source: entries of D rows become the identity's, entries in
    // D columns of the other rows zero (symmetric elimination)
    ctx->dirichlet = true;
    std::vector<uint8_t> em(s.n_pad, 0), drow(nrows, 0), dmesh(a.n, 0);
    for (int64_t i = 0; i < a.n; ++i) {
      drow[i] = a.dir[i];
      dmesh[ctx->perm.empty() ? i : ctx->perm[i]] = a.dir[i];
    }
    for (int64_t i = 0; i < a.n; ++i) {
      const int64_t sl = i / kWave, l = i % kWave, w = (s.ptr[sl + 1] - s.ptr[sl]) / kWave;
      for (int64_t k = 0; k < w; ++k) {
        const int64_t p = s.ptr[sl] + k * kWave + l;
        if (s.src[p] < 0) continue;
        const int32_t j = s.col[p];
        if (a.dir[i]) em[p] = j == i ? 2 : 1;
        else if (a.dir[j]) em[p] = 1;
      }
    }
    HZ_TRY(put(ctx, ctx->d_emask, em.data(), em.size()));
    HZ_TRY(put(ctx, ctx->d_dirrow, drow.data(), drow.size()));
    HZ_TRY(put(ctx, ctx->d_dirmesh, dmesh.data(), dmesh.size()));
  }
  // The load and the gradient kernels work on caller-ordered vectors: their
  // node ids go up in the mesh's own numbering.
  const std::vector<int32_t>& P = ctx->perm;
  auto to_mesh = [&](const std::vector<int32_t>& v) {
    std::vector<int32_t> o(v);
    if (!P.empty())
      for (int32_t& x : o) x = P[x];
    return o;
  };
  HZ_TRY(put(ctx, ctx->d_prow, to_mesh(a.prow).data(), a.prow.size()));
  HZ_TRY(put(ctx, ctx->d_pptr, a.pptr.data(), a.pptr.size()));
  HZ_TRY(put(ctx, ctx->d_pcol, to_mesh(a.pcol).data(), a.pcol.size()));
  HZ_TRY(put(ctx, ctx->d_pval, a.pval.data(), a.pval.size()));
  {
    std::vector<double> xyz(a.xyz);
    if (!P.empty())
      for (int64_t p = 0; p < a.n; ++p)
        for (int d = 0; d < 3; ++d) xyz[int64_t(P[p]) * 3 + d] = a.xyz[p * 3 + d];
    HZ_TRY(put(ctx, ctx->d_xyz, xyz.data(), xyz.size()));
  }
  HZ_TRY(put(ctx, ctx->d_hex, to_mesh(a.hex).data(), a.hex.size()));
  HZ_TRY(put(ctx, ctx->d_bface, to_mesh(a.bface).data(), a.bface.size()));
  HZ_TRY(put(ctx, ctx->d_btag, a.btag.data(), a.btag.size()));
  if (!P.empty()) HZ_TRY(put(ctx, ctx->d_perm, P.data(), P.size()));
  size_t before = ctx->d_A.bytes + ctx->d_d.bytes + ctx->d_dinv.bytes;
  HZ_TRY(ctx->d_A.ensure(sizeof(z_t) * s.n_pad));
  HZ_TRY(ctx->d_d.ensure(sizeof(z_t) * nrows));
  HZ_TRY(ctx->d_dinv.ensure(sizeof(z_t) * nrows));
  ctx->dev_bytes += int64_t(ctx->d_A.bytes + ctx->d_d.bytes + ctx->d_dinv.bytes) - int64_t(before);
  HZ_TRY(ctx_upload_params(ctx));
  return HZ_OK;
}

int ctx_single_seg(hz_ctx ctx, SegHost** out) {
  SegHost* S = ctx->single_seg.get();
  if (!S) {
    ctx->single_seg.reset(new SegHost());
    S = ctx->single_seg.get();
    S->nseg = 1;
    S->nrows = ctx->sell.n_rows;
    S->nblk = int(S->nrows / kBlock);
    S->seg_blk = {0, S->nblk};
    S->seg_n = {ctx->h.n};
    HZ_TRY(seg_upload(ctx, S, "single"));
  }
  *out = S;
  return HZ_OK;
}
