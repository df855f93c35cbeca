// Model files: hdmr_model_save / hdmr_model_load.
//
// Layout (native little-endian):
//   "HDMRASG1" (8 bytes), uint32 version = 1, int32 d, int32 m,
//   int32 n_components, double c0[m];
//   per component: int32 k, int32 dims[k], double weight, int64 npts,
//   uint8 levels[npts*k], uint32 indices[npts*k], double surpluses[npts*m]
// (rows in the model's internal order, as hdmr_export_component gives them).
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "hdmr_internal.h"

using namespace hdmr;

namespace {

constexpr char kMagic[8] = {'H', 'D', 'M', 'R', 'A', 'S', 'G', '1'};
constexpr uint32_t kVersion = 1;

struct FileCloser {
  void operator()(FILE *f) const {
    if (f) std::fclose(f);
  }
};
using File = std::unique_ptr<FILE, FileCloser>;

bool put(FILE *f, const void *p, size_t bytes) { return bytes == 0 || std::fwrite(p, 1, bytes, f) == bytes; }
bool get(FILE *f, void *p, size_t bytes) { return bytes == 0 || std::fread(p, 1, bytes, f) == bytes; }

}  // namespace

extern "C" {

int hdmr_model_save(const hdmr_model *model, const char *path) {
  clear_error();
  if (!model || !path) return fail(HDMR_EINVAL, "hdmr_model_save: null argument");
  File f(std::fopen(path, "wb"));
  if (!f) return fail(HDMR_EINVAL, std::string("cannot open '") + path + "' for writing");
  const int32_t d = model->d, m = model->m, nc = (int32_t)model->comps.size();
  bool ok = put(f.get(), kMagic, 8) && put(f.get(), &kVersion, 4) && put(f.get(), &d, 4) && put(f.get(), &m, 4) &&
            put(f.get(), &nc, 4) && put(f.get(), model->c0_h.data(), sizeof(double) * (size_t)m);
  std::vector<uint8_t> lv;
  std::vector<uint32_t> ix;
  std::vector<double> al;
  for (int32_t s = 0; ok && s < nc; ++s) {
    int64_t n = 0;
    int32_t k = 0, dims[KMAX] = {0, 0, 0, 0};
    double w = 0.0;
    int rc = hdmr_export_component(model, s, &n, &k, dims, nullptr, nullptr, nullptr, &w);
    if (rc) return rc;
    lv.resize((size_t)(n * k));
    ix.resize((size_t)(n * k));
    al.resize((size_t)(n * m));
    rc = hdmr_export_component(model, s, &n, &k, dims, lv.data(), ix.data(), al.data(), &w);
    if (rc) return rc;
    ok = put(f.get(), &k, 4) && put(f.get(), dims, sizeof(int32_t) * (size_t)k) && put(f.get(), &w, 8) &&
         put(f.get(), &n, 8) && put(f.get(), lv.data(), lv.size()) && put(f.get(), ix.data(), 4 * ix.size()) &&
         put(f.get(), al.data(), 8 * al.size());
  }
  if (!ok || std::fflush(f.get()) != 0) return fail(HDMR_EINVAL, std::string("write to '") + path + "' failed");
  return HDMR_OK;
}

namespace {

// Size of the open file (bytes), or -1.
int64_t file_size(std::FILE *f) {
  const long at = std::ftell(f);
  if (at < 0 || std::fseek(f, 0, SEEK_END) != 0) return -1;
  const long end = std::ftell(f);
  if (std::fseek(f, at, SEEK_SET) != 0) return -1;
  return end;
}

int model_load(const char *path, hdmr_model **out) {
  File f(std::fopen(path, "rb"));
  if (!f) return fail(HDMR_EINVAL, std::string("cannot open '") + path + "'");
  const int64_t total = file_size(f.get());
  if (total < 0) return fail(HDMR_EINVAL, std::string("cannot size '") + path + "'");
  char magic[8];
  uint32_t version = 0;
  int32_t d = 0, m = 0, nc = 0;
  if (!get(f.get(), magic, 8) || std::memcmp(magic, kMagic, 8) != 0)
    return fail(HDMR_EINVAL, std::string("'") + path + "' is not a model file");
  if (!get(f.get(), &version, 4) || version != kVersion)
    return fail(HDMR_EUNSUPPORTED, "unsupported model file version");
  if (!get(f.get(), &d, 4) || !get(f.get(), &m, 4) || !get(f.get(), &nc, 4) || d < 1 || m < 1 || nc < 0)
    return fail(HDMR_EINVAL, "corrupt model file header");
  // every count is checked against the bytes left in the file before any
  // buffer is sized from it (no overflow: each factor is bounded first)
  int64_t left = total - std::ftell(f.get());
  if ((int64_t)m > left / 8) return fail(HDMR_EINVAL, "corrupt model file header (m exceeds the file)");
  if ((int64_t)nc > left / 20) return fail(HDMR_EINVAL, "corrupt model file header (components exceed the file)");
  std::vector<double> c0((size_t)m);
  if (!get(f.get(), c0.data(), 8 * (size_t)m)) return fail(HDMR_EINVAL, "truncated model file");
  std::vector<int32_t> offsets(1, 0), dims;
  std::vector<int64_t> npts;
  std::vector<double> weights, al;
  std::vector<uint8_t> lv;
  std::vector<uint32_t> ix;
  for (int32_t s = 0; s < nc; ++s) {
    int32_t k = 0;
    double w = 0.0;
    int64_t n = 0;
    if (!get(f.get(), &k, 4) || k < 1 || k > KMAX) return fail(HDMR_EINVAL, "corrupt component header");
    int32_t cd[KMAX];
    if (!get(f.get(), cd, 4 * (size_t)k) || !get(f.get(), &w, 8) || !get(f.get(), &n, 8) || n < 0)
      return fail(HDMR_EINVAL, "corrupt component header");
    left = total - std::ftell(f.get());
    // a row takes k level bytes, 4 k index bytes and 8 m surplus bytes
    const int64_t row_bytes = 5 * (int64_t)k + 8 * (int64_t)m;
    if (n > left / row_bytes) return fail(HDMR_EINVAL, "corrupt component header (rows exceed the file)");
    dims.insert(dims.end(), cd, cd + k);
    offsets.push_back(offsets.back() + k);
    npts.push_back(n);
    weights.push_back(w);
    const size_t l0 = lv.size(), a0 = al.size();
    lv.resize(l0 + (size_t)(n * k));
    ix.resize(l0 + (size_t)(n * k));
    al.resize(a0 + (size_t)(n * m));
    if (!get(f.get(), lv.data() + l0, (size_t)(n * k)) || !get(f.get(), ix.data() + l0, 4 * (size_t)(n * k)) ||
        !get(f.get(), al.data() + a0, 8 * (size_t)(n * m)))
      return fail(HDMR_EINVAL, "truncated model file");
  }
  return hdmr_model_from_surpluses(d, m, c0.data(), nc, offsets.data(), dims.data(), npts.data(), lv.data(),
                                   ix.data(), al.data(), weights.data(), out);
}

}  // namespace

int hdmr_model_load(const char *path, hdmr_model **out) {
  clear_error();
  if (!path || !out) return fail(HDMR_EINVAL, "hdmr_model_load: null argument");
  *out = nullptr;
  try {
    return model_load(path, out);
  } catch (const std::bad_alloc &) {
    return fail(HDMR_ENOMEM, "hdmr_model_load: host allocation failed");
  } catch (...) {
    return fail(HDMR_EINVAL, "hdmr_model_load: corrupt model file");
  }
}

}  // extern "C"
