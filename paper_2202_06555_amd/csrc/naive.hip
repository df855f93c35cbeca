// The naive evaluation of eq (3.16): every term of the double sum over the
// retained index sets u and their subsets v is its own sparse-grid
// interpolation of the cut function g_v = f(xbar \ x_v), so cut interpolants
// shared by several u are recomputed once per u (the direct implementation
// that Sec. 4.1 contrasts with the regrouped form a(x)^T b of eq (4.2)).
// The expanded model holds one component per (u, v != empty) term, with
// weight (-1)^(|u|-|v|) and a copy of g_v's grid and surpluses; the empty-set
// terms fold into c0 = f(xbar) sum_{u in U + {empty}} (-1)^|u|.  It is
// evaluated by the same kernels as every other model.
#include <map>
#include <vector>

#include "hdmr_internal.h"

using namespace hdmr;

extern "C" {

int hdmr_model_naive(const hdmr_model *src, const double *f_anchor, hdmr_model **out) {
  clear_error();
  if (!src || !f_anchor || !out) return fail(HDMR_EINVAL, "hdmr_model_naive: null argument");
  *out = nullptr;
  const int32_t nc = (int32_t)src->comps.size(), m = src->m;
  struct Grid {
    int64_t n = 0;
    int32_t k = 0;
    int32_t dims[KMAX] = {0, 0, 0, 0};
    std::vector<uint8_t> lv;
    std::vector<uint32_t> ix;
    std::vector<double> al;
  };
  std::vector<Grid> g((size_t)nc);
  std::map<std::vector<int32_t>, int32_t> where;
  double wt = 0.0;
  for (int32_t c = 0; c < nc; ++c) {
    Grid &G = g[(size_t)c];
    int rc = hdmr_export_component(src, c, &G.n, &G.k, G.dims, nullptr, nullptr, nullptr, &wt);
    if (rc) return rc;
    G.lv.resize((size_t)(G.n * G.k));
    G.ix.resize((size_t)(G.n * G.k));
    G.al.resize((size_t)(G.n * m));
    rc = hdmr_export_component(src, c, &G.n, &G.k, G.dims, G.lv.data(), G.ix.data(), G.al.data(), &wt);
    if (rc) return rc;
    where[std::vector<int32_t>(G.dims, G.dims + G.k)] = c;
  }
  // terms (u, v): v runs over the nonempty subsets of u (bit masks over u's
  // dimensions); the sign counts the dimensions of u outside v
  std::vector<int32_t> term_comp;
  std::vector<double> term_sign;
  double c0_sign = 1.0;  // the empty set itself
  for (int32_t c = 0; c < nc; ++c) {
    const Grid &U = g[(size_t)c];
    c0_sign += (U.k % 2) ? -1.0 : 1.0;
    for (uint32_t mask = 1; mask < (1u << U.k); ++mask) {
      std::vector<int32_t> v;
      for (int32_t q = 0; q < U.k; ++q)
        if (mask & (1u << q)) v.push_back(U.dims[q]);
      const auto it = where.find(v);
      if (it == where.end())
        return fail(HDMR_EINVAL, "hdmr_model_naive: the components are not closed under subsets (component " +
                                     std::to_string(c) + " lacks a subset)");
      term_comp.push_back(it->second);
      term_sign.push_back(((U.k - (int32_t)v.size()) % 2) ? -1.0 : 1.0);
    }
  }
  std::vector<double> c0((size_t)m);
  for (int32_t o = 0; o < m; ++o) c0[(size_t)o] = c0_sign * f_anchor[o];
  std::vector<int32_t> offs(1, 0), dims;
  std::vector<int64_t> npts;
  std::vector<uint8_t> lv;
  std::vector<uint32_t> ix;
  std::vector<double> al, w;
  for (size_t t = 0; t < term_comp.size(); ++t) {
    const Grid &G = g[(size_t)term_comp[t]];
    dims.insert(dims.end(), G.dims, G.dims + G.k);
    offs.push_back(offs.back() + G.k);
    npts.push_back(G.n);
    lv.insert(lv.end(), G.lv.begin(), G.lv.end());
    ix.insert(ix.end(), G.ix.begin(), G.ix.end());
    al.insert(al.end(), G.al.begin(), G.al.end());
    w.push_back(term_sign[t]);
  }
  return hdmr_model_from_surpluses(src->d, m, c0.data(), (int32_t)term_comp.size(), offs.data(), dims.data(),
                                   npts.data(), lv.data(), ix.data(), al.data(), w.data(), out);
}

}  // extern "C"
