// Segment layouts and segmented reductions shared by the solvers.
#include "ops.h"

namespace {

template <typename T>
__global__ void __launch_bounds__(kBlock) k_norm_part(Seg L, const cx<T>* __restrict__ x, double* part) {
  SumTile t = tile_of_sums(L);
  double q[1] = {norm2(ccast<double>(x[t.row]))};
  store_partials<1>(q, part, t);
}

__global__ void k_seg_fin1(Seg L, const double* part, double* out) {
  int s = blockIdx.x;
  double o[1];
  seg_sums<1>(L, part, s, o);
  if (threadIdx.x == 0) out[s] = o[0];
}

// r = f - A u (FP64), partial ||r||^2; per storage form F of A.
template <int F>
__global__ void __launch_bounds__(kBlock) k_true_resid(Seg L, SellOp<double> A, const z_t* __restrict__ f,
                                                       const z_t* __restrict__ u, z_t* __restrict__ r,
                                                       double* part) {
  SumTile t = tile_of_sums(L);
  z_t v = f[t.row] - sell_row_form<F>(A, t.row, u);
  if (r) r[t.row] = v;
  double q[1] = {norm2(v)};
  store_partials<1>(q, part, t);
}

int fetch_seg(hz_ctx ctx, const SegHost& S, const double* dev, std::vector<double>* out) {
  void* hp = nullptr;
  HZ_TRY(ctx_pinned(ctx, sizeof(double) * S.nseg, &hp));
  HZ_HIP(hipMemcpyAsync(hp, dev, sizeof(double) * S.nseg, hipMemcpyDeviceToHost, ctx->stream));
  HZ_HIP(hipStreamSynchronize(ctx->stream));
  out->assign(static_cast<double*>(hp), static_cast<double*>(hp) + S.nseg);
  return HZ_OK;
}

}  // namespace

template <typename T>
int seg_norm2_t(hz_ctx ctx, const SegHost& S, const cx<T>* x, std::vector<double>* out) {
  int rc = 0;
  DevBuf* part = ctx->buf("segn.part", sizeof(double) * S.nblk, &rc);
  if (rc) return rc;
  DevBuf* res = ctx->buf("segn.out", sizeof(double) * S.nseg, &rc);
  if (rc) return rc;
  k_norm_part<T><<<S.nblk, kBlock, 0, ctx->stream>>>(S.dev, x, part->as<double>());
  k_seg_fin1<<<S.nseg, kFinBlock, 0, ctx->stream>>>(S.dev, part->as<double>(), res->as<double>());
  HZ_HIP(hipGetLastError());
  return fetch_seg(ctx, S, res->as<double>(), out);
}
template int seg_norm2_t<double>(hz_ctx, const SegHost&, const z_t*, std::vector<double>*);
template int seg_norm2_t<float>(hz_ctx, const SegHost&, const c_t*, std::vector<double>*);

int true_residual(hz_ctx ctx, const SegHost& S, const SellOp<double>& A, const z_t* f, const z_t* u,
                  z_t* r, std::vector<double>* rr) {
  int rc = 0;
  DevBuf* part = ctx->buf("tres.part", sizeof(double) * S.nblk, &rc);
  if (rc) return rc;
  DevBuf* res = ctx->buf("tres.out", sizeof(double) * S.nseg, &rc);
  if (rc) return rc;
  if (A.val) k_true_resid<kFormComplex><<<S.nblk, kBlock, 0, ctx->stream>>>(S.dev, A, f, u, r, part->as<double>());
  else if (A.st) k_true_resid<kFormStencil><<<S.nblk, kBlock, 0, ctx->stream>>>(S.dev, A, f, u, r, part->as<double>());
  else k_true_resid<kFormSplit><<<S.nblk, kBlock, 0, ctx->stream>>>(S.dev, A, f, u, r, part->as<double>());
  k_seg_fin1<<<S.nseg, kFinBlock, 0, ctx->stream>>>(S.dev, part->as<double>(), res->as<double>());
  HZ_HIP(hipGetLastError());
  return fetch_seg(ctx, S, res->as<double>(), rr);
}

int seg_upload(hz_ctx ctx, SegHost* S, const std::string& tag) {
  int rc = 0;
  // the segments tile the blocks (the finalize kernels rely on it)
  if (int(S->seg_blk.size()) != S->nseg + 1 || S->seg_blk.front() != 0 || S->seg_blk.back() != S->nblk)
    return hz_fail(HZ_ERR_INVALID, "segment table does not tile the %d blocks", S->nblk);
  std::vector<int> blk_seg(S->nblk);
  for (int s = 0; s < S->nseg; ++s)
    for (int b = S->seg_blk[s]; b < S->seg_blk[s + 1]; ++b) blk_seg[b] = s;
  DevBuf* a = ctx->buf(tag + ".blk_seg", sizeof(int) * S->nblk, &rc);
  if (rc) return rc;
  DevBuf* b = ctx->buf(tag + ".seg_blk", sizeof(int) * (S->nseg + 1), &rc);
  if (rc) return rc;
  HZ_HIP(hipMemcpy(a->p, blk_seg.data(), sizeof(int) * S->nblk, hipMemcpyHostToDevice));
  HZ_HIP(hipMemcpy(b->p, S->seg_blk.data(), sizeof(int) * (S->nseg + 1), hipMemcpyHostToDevice));
  S->dev.nseg = S->nseg;
  S->dev.nblk = S->nblk;
  S->dev.nrows = S->nrows;
  S->dev.blk_seg = a->as<int>();
  S->dev.seg_blk = b->as<int>();
  return HZ_OK;
}
