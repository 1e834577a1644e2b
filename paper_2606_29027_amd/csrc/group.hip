// Host side of the grouped launches: descriptors and block offsets staged
// in pinned memory, one upload per flush, launches issued in order.
#include <algorithm>
#include <cstring>

#include "group.h"

namespace slar {

namespace {
constexpr size_t GQ_ALIGN = 256;
size_t gq_align(size_t x) { return (x + GQ_ALIGN - 1) & ~(GQ_ALIGN - 1); }
}  // namespace

const void* GroupQueue::stage(const void* src, size_t bytes) {
  const size_t off = gq_align(used_);
  if (off + bytes > cap_) {
    overflow_ = true;
    return nullptr;
  }
  std::memcpy(h_ + off, src, bytes);
  used_ = off + bytes;
  return d_ + off;
}

template <class D>
bool GroupQueue::push(const std::vector<D>& descs, const std::vector<int>& first, const D** dd, const int** df) {
  *dd = (const D*)stage(descs.data(), sizeof(D) * descs.size());
  *df = (const int*)stage(first.data(), sizeof(int) * first.size());
  return *dd && *df;
}

hipError_t GroupQueue::gemm(bool ta, bool tb, const std::vector<GemmArgs>& p) {
  std::vector<GemmDesc> ds;
  std::vector<int> first;
  int nb = 0;
  for (const GemmArgs& a : p) {
    if (a.M <= 0 || a.N <= 0 || a.batch <= 0) continue;   // nothing to compute (as gemm_f64)
    if (a.K < 0) return hipErrorInvalidValue;
    GemmDesc g{};
    g.M = a.M; g.N = a.N; g.K = a.K;
    g.tm = (a.M + 63) / 64; g.tn = (a.N + 63) / 64;
    g.alpha = a.alpha; g.beta = a.beta;
    g.A = a.A; g.B = a.B; g.C = a.C;
    g.lda = a.lda; g.ldb = a.ldb; g.ldc = a.ldc;
    g.sA = a.sA; g.sB = a.sB; g.sC = a.sC;
    const long long blocks = (long long)g.tm * g.tn * a.batch;
    if (nb + blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    ds.push_back(g);
    first.push_back(nb);
    nb += (int)blocks;
  }
  if (ds.empty()) return hipSuccess;
  const GemmDesc* dd;
  const int* df;
  if (!push(ds, first, &dd, &df)) return hipErrorOutOfMemory;
  const int nd = (int)ds.size();
  then([=](hipStream_t s) { return gemm_group_launch(s, ta, tb, dd, df, nd, nb); });
  return hipSuccess;
}

hipError_t GroupQueue::gram(const std::vector<GramArgs>& p) {
  // per problem the block count of the one-problem call; MT 4 (k <= 64) and
  // MT 8 problems in separate part launches, one sum launch for all
  std::vector<GramDesc> d4, d8, dall;
  std::vector<int> f4, f8, fs;
  int n4 = 0, n8 = 0, ns = 0;
  for (const GramArgs& a : p) {
    if (a.k < 1 || a.k > 128 || a.n < 1) return hipErrorInvalidValue;
    const int nchunk = (a.n + 31) / 32;
    int nblk = std::min(nchunk, 128);
    while (nblk > 1 && (size_t)nblk * a.k * a.k > a.part_cap) nblk /= 2;
    if ((size_t)nblk * a.k * a.k > a.part_cap) return hipErrorInvalidValue;
    GramDesc g{};
    g.k = a.k; g.n = a.n; g.nblk = nblk; g.mode2 = a.mode2;
    g.A = a.A; g.lda = a.lda; g.nb = a.nb; g.r = a.r;
    g.part = a.part; g.G = a.G;
    if (a.k <= 64) { d4.push_back(g); f4.push_back(n4); n4 += nblk; }
    else { d8.push_back(g); f8.push_back(n8); n8 += nblk; }
    dall.push_back(g);
    fs.push_back(ns);
    ns += (a.k * a.k + 63) / 64;
  }
  if (dall.empty()) return hipSuccess;
  const GramDesc *p4 = nullptr, *p8 = nullptr, *pa = nullptr;
  const int *q4 = nullptr, *q8 = nullptr, *qa = nullptr;
  if (!d4.empty() && !push(d4, f4, &p4, &q4)) return hipErrorOutOfMemory;
  if (!d8.empty() && !push(d8, f8, &p8, &q8)) return hipErrorOutOfMemory;
  if (!push(dall, fs, &pa, &qa)) return hipErrorOutOfMemory;
  const int c4 = (int)d4.size(), c8 = (int)d8.size(), ca = (int)dall.size();
  then([=](hipStream_t s) {
    hipError_t e = gram_part_group_launch(s, false, p4, q4, c4, n4);
    if (e == hipSuccess) e = gram_part_group_launch(s, true, p8, q8, c8, n8);
    if (e == hipSuccess) e = gram_sum_group_launch(s, pa, qa, ca, ns);
    return e;
  });
  return hipSuccess;
}

hipError_t GroupQueue::copy2d(const std::vector<CopyDesc>& p) {
  std::vector<CopyDesc> ds;
  std::vector<int> first;
  int nb = 0;
  for (const CopyDesc& c : p) {
    const long long n = (long long)c.rows * c.cols;
    if (n <= 0) continue;
    ds.push_back(c);
    first.push_back(nb);
    nb += (int)((n + 255) / 256);
  }
  if (ds.empty()) return hipSuccess;
  const CopyDesc* dd;
  const int* df;
  if (!push(ds, first, &dd, &df)) return hipErrorOutOfMemory;
  const int nd = (int)ds.size();
  then([=](hipStream_t s) { return copy2d_group_launch(s, dd, df, nd, nb); });
  return hipSuccess;
}

hipError_t GroupQueue::sign_fix(const std::vector<SignArgs>& p) {
  std::vector<SignDesc> ds;
  std::vector<int> first;
  int nb = 0;
  for (const SignArgs& a : p) {
    if (a.cols <= 0) continue;
    SignDesc g{};
    g.rows = a.rows; g.cols = a.cols; g.lda = a.lda; g.ldb = a.ldb; g.rowsB = a.rowsB;
    g.A = a.A; g.B = a.B;
    ds.push_back(g);
    first.push_back(nb);
    nb += a.cols;
  }
  if (ds.empty()) return hipSuccess;
  const SignDesc* dd;
  const int* df;
  if (!push(ds, first, &dd, &df)) return hipErrorOutOfMemory;
  const int nd = (int)ds.size();
  then([=](hipStream_t s) { return sign_fix_group_launch(s, dd, df, nd, nb); });
  return hipSuccess;
}

hipError_t GroupQueue::sign_fix_tall(const std::vector<SignArgs>& p) {
  // the choice of sign_fix_tall per problem: three coalesced passes, or the
  // one-pass form for wide matrices or too little scratch
  std::vector<SignArgs> one;
  std::vector<SignDesc> ds;
  std::vector<int> fp, fd, fa;
  int np = 0, ndc = 0, na = 0;
  for (const SignArgs& a : p) {
    if (a.cols <= 0) continue;
    const int nb = std::min(256, std::max(1, (a.rows + 63) / 64));
    const int rb = (a.rows + nb - 1) / nb;
    if (a.cols > 64 || !a.scratch || (size_t)(nb + 1) * a.cols > a.scratch_elems) {
      one.push_back(a);
      continue;
    }
    SignDesc g{};
    g.rows = a.rows; g.cols = a.cols; g.lda = a.lda; g.ldb = a.ldb; g.rowsB = a.rowsB;
    g.rb = rb; g.nb = nb;
    g.A = a.A; g.B = a.B; g.part = a.scratch;
    const long long elems = (long long)a.rows * a.cols + (a.B ? (long long)a.rowsB * a.cols : 0);
    ds.push_back(g);
    fp.push_back(np); np += nb;
    fd.push_back(ndc); ndc += a.cols;
    fa.push_back(na); na += (int)((elems + 255) / 256);
  }
  if (!one.empty()) {
    const hipError_t e = sign_fix(one);
    if (e != hipSuccess) return e;
  }
  if (ds.empty()) return hipSuccess;
  const SignDesc* dd;
  const int *qp, *qd, *qa;
  dd = (const SignDesc*)stage(ds.data(), sizeof(SignDesc) * ds.size());
  qp = (const int*)stage(fp.data(), sizeof(int) * fp.size());
  qd = (const int*)stage(fd.data(), sizeof(int) * fd.size());
  qa = (const int*)stage(fa.data(), sizeof(int) * fa.size());
  if (!dd || !qp || !qd || !qa) return hipErrorOutOfMemory;
  const int nd = (int)ds.size();
  then([=](hipStream_t s) {
    hipError_t e = sign_part_group_launch(s, dd, qp, nd, np);
    if (e == hipSuccess) e = sign_decide_group_launch(s, dd, qd, nd, ndc);
    if (e == hipSuccess) e = sign_apply_group_launch(s, dd, qa, nd, na);
    return e;
  });
  return hipSuccess;
}

hipError_t GroupQueue::scale(const std::vector<ScaleDesc>& p) {
  std::vector<ScaleDesc> ds;
  std::vector<int> first;
  int nb = 0;
  for (const ScaleDesc& a : p) {
    const long long n = a.diag ? (long long)a.r * a.r : (long long)a.k * a.r;
    if (n <= 0) continue;
    ds.push_back(a);
    first.push_back(nb);
    nb += (int)((n + 255) / 256);
  }
  if (ds.empty()) return hipSuccess;
  const ScaleDesc* dd;
  const int* df;
  if (!push(ds, first, &dd, &df)) return hipErrorOutOfMemory;
  const int nd = (int)ds.size();
  then([=](hipStream_t s) { return scale_group_launch(s, dd, df, nd, nb); });
  return hipSuccess;
}

// one launch over problems whose block count is count(desc) each
template <class D, class C, class L>
static hipError_t simple_group(GroupQueue& q, const std::vector<D>& p, C count, L launch) {
  std::vector<D> ds;
  std::vector<int> first;
  long long nb = 0;
  for (const D& a : p) {
    const long long c = count(a);
    if (c <= 0) continue;
    ds.push_back(a);
    first.push_back((int)nb);
    nb += c;
  }
  if (ds.empty()) return hipSuccess;
  if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
  const D* dd = (const D*)q.stage(ds.data(), sizeof(D) * ds.size());
  const int* df = (const int*)q.stage(first.data(), sizeof(int) * first.size());
  if (!dd || !df) return hipErrorOutOfMemory;
  const int nd = (int)ds.size(), nbi = (int)nb;
  q.then([=](hipStream_t s) { return launch(s, dd, df, nd, nbi); });
  return hipSuccess;
}

hipError_t GroupQueue::lines(const std::vector<LineDesc>& p) {
  std::vector<LineDesc> fft, dft;
  for (const LineDesc& a : p) (a.logL >= 1 ? fft : dft).push_back(a);
  auto count = [](const LineDesc& a) { return (long long)(a.axis == 1 ? a.n0 : a.n1) * a.B; };
  HIP_CHK(simple_group(*this, fft, count, [](hipStream_t s, const LineDesc* d, const int* f, int nd, int nb) {
    return line_group_launch(s, true, d, f, nd, nb);
  }));
  return simple_group(*this, dft, count, [](hipStream_t s, const LineDesc* d, const int* f, int nd, int nb) {
    return line_group_launch(s, false, d, f, nd, nb);
  });
}

hipError_t GroupQueue::field(const std::vector<FieldDesc>& p) {
  auto count = [](const FieldDesc& a) {
    const long long n = a.op == FIELD_SYMBOL ? (long long)a.Nx * a.nvec : a.n;
    return (n + 255) / 256;
  };
  return simple_group(*this, p, count, [](hipStream_t s, const FieldDesc* d, const int* f, int nd, int nb) {
    return field_group_launch(s, d, f, nd, nb);
  });
}

hipError_t GroupQueue::sums(const std::vector<SumDesc>& p) {
  auto count = [](const SumDesc& a) { return ((long long)a.M * a.N + 255) / 256; };
  return simple_group(*this, p, count, [](hipStream_t s, const SumDesc* d, const int* f, int nd, int nb) {
    return sum_group_launch(s, d, f, nd, nb);
  });
}

hipError_t GroupQueue::flush(hipStream_t s) {
  if (overflow_) return hipErrorOutOfMemory;
  if (used_ > flushed_) {
    const hipError_t e = hipMemcpyAsync(d_ + flushed_, h_ + flushed_, used_ - flushed_, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    flushed_ = used_;
  }
  for (auto& op : ops_) {
    const hipError_t e = op(s);
    if (e != hipSuccess) {
      ops_.clear();
      return e;
    }
  }
  ops_.clear();
  return hipSuccess;
}

}  // namespace slar
