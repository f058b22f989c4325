// Perturbative triples correction E_(T) of the M_s = 1 high-spin determinant
// (standard single-reference (T) expression in spin orbitals; the paper names
// triples extensions only as other work).
//
// Layout and flow:
//  * once per context: the integrals <ei||bc> of every occupied spin orbital
//    i, <jk||bc> and <ma||jk>, assembled from spatial DF products (FP64 MFMA
//    GEMMs over the auxiliary index) with the spin selection rules applied
//    elementwise.  The <ei||bc> rows of i share a slab with the amplitude rows
//    t_im^bc (written per call), ordered by spin so that for each spin s the
//    rows [virtual e of spin s | occupied m of spin s] are contiguous: the two
//    sums of the connected numerator become one GEMM over n = v_s + o_s;
//  * per call: the packed amplitudes unpacked to spin orbitals, then for each
//    occupied triple i < j < k
//      Zt[a][bc] = P(i/jk) [sum_e t_jk^ae <ei||bc> - sum_m t_im^bc <ma||jk>]
//    as one FP64 GEMM per spin of a, written once into one n_vir x n_vir^2
//    array: its K runs over the orders of (i, j, k) that spin conservation
//    allows for that spin (up to three segments of n), each segment reading
//    the slab rows of its own x; then one pass over a < b < c, tiled through
//    LDS so that Zt[c][b][a]
//    is read along a, that forms N^c = P(a/bc) Zt, the disconnected numerator
//    and the denominator and reduces the three energy parts in a fixed order.
#include <vector>

#include "ops.h"

namespace dcsd {

namespace {
// Device array for the set-up only, freed when it leaves scope.
struct Tmp {
  double* p = nullptr;
  explicit Tmp(int64_t n) {
    if (hipMalloc(&p, (size_t)std::max<int64_t>(n, 1) * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      throw std::bad_alloc();
    }
  }
  ~Tmp() {
    if (p) (void)hipFree(p);
  }
  Tmp(const Tmp&) = delete;
  Tmp& operator=(const Tmp&) = delete;
};
}  // namespace

void Ctx::triples(const double* T, dcsd_triples_energy* out, double* contrib) {
  if (!method_hs(cfg.method))
    throw ArgError("the triples correction is defined for the high-spin methods (DCSD_METHOD_HS_*) only");
  TriDims d;
  d.oa = os[0];
  d.ob = os[1];
  d.va = vs[0];
  d.vb = vs[1];
  d.n = n;
  d.nU = n - os[1];
  const int64_t nO = d.nO(), nV = d.nV(), nU = d.nU, NA = naux, oa = d.oa;
  const int64_t nV2 = nV * nV, nV3 = nV2 * nV;
  const int64_t ntrip = nO * (nO - 1) * (nO - 2) / 6;
  if (!tri.ready) {
    // (a call that failed part-way, e.g. out of memory, keeps what it had allocated for the next)
    auto once = [&](double*& p, int64_t count) {
      if (!p) p = alloc(count);
    };
    once(tri.t1so, nO * nV);
    once(tri.fov, nO * nV);
    once(tri.fo, nO);
    once(tri.fv, nV);
    once(tri.t2so, nO * nO * nV2);
    once(tri.oovv, nO * nO * nV2);
    once(tri.Q, nO * nO * nV * nO);
    once(tri.I, nO * d.slab_rows() * nV2);
    once(tri.Aop, nV * (3 * (int64_t)n + 1));
    once(tri.Zt, nV3);
    once(tri.part, 3 * tri_energy_blocks(d));
    once(tri.out, std::max<int64_t>(4 * ntrip, 4));
    // spatial factor blocks: U x U, occupied x U, occupied x occupied, U x occupied
    const double* Bsp = Bs[0];
    const int64_t ob = d.ob;
    Tmp BU(NA * nU * nU), BO(NA * oa * nU), BOO(NA * oa * oa), BVO(NA * nU * oa);
    copyN(BU.p, Bsp + ob * n + ob, {NA, nU, nU}, {nU * nU, nU, 1}, {n2, n, 1}, 1.0, 0.0, s);
    copyN(BO.p, Bsp + ob, {NA, oa, nU}, {oa * nU, nU, 1}, {n2, n, 1}, 1.0, 0.0, s);
    copyN(BOO.p, Bsp, {NA, oa, oa}, {oa * oa, oa, 1}, {n2, n, 1}, 1.0, 0.0, s);
    copyN(BVO.p, Bsp + ob * n, {NA, nU, oa}, {nU * oa, oa, 1}, {n2, n, 1}, 1.0, 0.0, s);
    {
      // S[(e,b)][(x,c)] = (eb|xc) -> <ex||bc>
      Tmp S(nU * nU * oa * nU);
      G(nU * nU, oa * nU, NA).A(BU.p, nU * nU, true).B(BO.p, oa * nU, true).C(S.p, oa * nU).run(*this);
      tri_assemble_vovv(tri.I, S.p, d, s);
      DCSD_HIP(hipStreamSynchronize(s));
    }
    {
      // S2[(j,b)][(k,c)] = (jb|kc) -> <jk||bc>;  S3[(m,y)][(a,z)] = (my|az) -> <ma||yz>
      Tmp S2(oa * nU * oa * nU), S3(oa * oa * nU * oa);
      G(oa * nU, oa * nU, NA).A(BO.p, oa * nU, true).B(BO.p, oa * nU, true).C(S2.p, oa * nU).run(*this);
      tri_assemble_oovv(tri.oovv, S2.p, d, s);
      G(oa * oa, nU * oa, NA).A(BOO.p, oa * oa, true).B(BVO.p, nU * oa, true).C(S3.p, nU * oa).run(*this);
      tri_assemble_ovoo(tri.Q, S3.p, d, s);
      DCSD_HIP(hipStreamSynchronize(s));
    }
    tri.ready = true;
  }
  tri_unpack(tri.t1so, tri.t2so, tri.fo, tri.fv, tri.fov, T, f[0], f[1], L, d, s);
  // amplitude rows t_xm^bc of every slab x (occupied m of each spin after that spin's virtuals)
  const int64_t R = d.slab_rows();
  copyN(tri.I + (int64_t)d.row_m(0) * nV2, tri.t2so, {nO, oa, nV2}, {R * nV2, nV2, 1}, {nO * nV2, nV2, 1}, 1.0, 0.0,
        s);
  copyN(tri.I + (int64_t)d.row_m(d.oa) * nV2, tri.t2so + oa * nV2, {nO, (int64_t)d.ob, nV2}, {R * nV2, nV2, 1},
        {nO * nV2, nV2, 1}, 1.0, 0.0, s);

  const int64_t off_v[2] = {0, d.va}, nvs[2] = {d.va, d.vb}, row_e[2] = {0, (int64_t)d.va + d.oa};
  const int64_t lda3 = 3 * (int64_t)n + ((3 * n) & 1);  // even, with a zero column after 3n
  int64_t t = 0;
  for (int i = 0; i < nO; ++i)
    for (int j = i + 1; j < nO; ++j)
      for (int k = j + 1; k < nO; ++k, ++t) {
        // P(i/jk): (x; y z) = (i; j k), (j; i k), (k; j i) with signs +, -, - (in the A operand).
        // Spin conservation: t_yz^{ae} and <ma||yz> need s(e) = s(m) = s(y) + s(z) - s(a); the
        // orders allowed for a of spin sa form the K segments of one product per spin, each
        // segment against the slab rows of its own x.
        const int xs[3] = {i, j, k}, ys[3] = {j, i, j}, zs[3] = {k, k, i};
        TriSegs g;
        int seg_se[2][3] = {};
        for (int sa = 0; sa < 2; ++sa)
          for (int p = 0; p < 3 && nvs[sa] > 0; ++p) {
            const int se = (ys[p] >= d.oa) + (zs[p] >= d.oa) - sa;
            if (se < 0 || se > 1) continue;
            seg_se[sa][g.nseg[sa]] = se;
            g.p[sa][g.nseg[sa]++] = p;
          }
        tri_operand_a(tri.Aop, lda3, tri.t2so, tri.Q, i, j, k, g, d, s);
        for (int sa = 0; sa < 2; ++sa) {
          if (nvs[sa] == 0) continue;
          double* Zs = tri.Zt + off_v[sa] * nV2;
          if (g.nseg[sa] == 0) {
            fill(Zs, 0.0, nvs[sa] * nV2, s);
            continue;
          }
          const double* As = tri.Aop + off_v[sa] * lda3;
          const double* bs[3] = {nullptr, nullptr, nullptr};
          for (int q = 0; q < g.nseg[sa]; ++q) bs[q] = tri.I + (xs[g.p[sa][q]] * R + row_e[seg_se[sa][q]]) * nV2;
          if (gemm_f64_bseg(nvs[sa], nV2, n, g.nseg[sa], As, lda3, bs, nV2, Zs, nV2, 1.0, 0.0, s)) continue;
          for (int q = 0; q < g.nseg[sa]; ++q)  // shapes the segmented product does not take
            G(nvs[sa], nV2, n).A(As + q * n, lda3, false).B(bs[q], nV2, true).C(Zs, nV2).ab(1.0, q ? 1.0 : 0.0).run(*this);
        }
        tri_energy(tri.out + 4 * t, tri.part, tri.Zt, tri.t1so, tri.t2so, tri.oovv, tri.fo, tri.fv, tri.fov, i, j, k,
                   d, s);
      }
  std::vector<double> h((size_t)std::max<int64_t>(4 * ntrip, 4), 0.0);
  if (ntrip > 0)
    DCSD_HIP(hipMemcpyAsync(h.data(), tri.out, 4 * ntrip * sizeof(double), hipMemcpyDeviceToHost, s));
  if (contrib && ntrip > 0) copyN(contrib, tri.out + 3, {ntrip}, {1}, {4}, 1.0, 0.0, s);
  DCSD_HIP(hipStreamSynchronize(s));
  dcsd_triples_energy e{};
  for (int64_t q = 0; q < ntrip; ++q) {
    e.e_t4 += h[4 * q + 0];
    e.e_st5 += h[4 * q + 1];
    e.e_dt += h[4 * q + 2];
  }
  e.e_t = e.e_t4 + e.e_st5 + e.e_dt;
  e.triples = ntrip;
  *out = e;
}

}  // namespace dcsd
