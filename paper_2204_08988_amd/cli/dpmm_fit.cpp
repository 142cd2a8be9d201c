// dpmm_fit: the command-line run of the sampler (the paper's command-line
// interface, Sec. 3.4) over the C ABI of libdpmm.so.
//
//   dpmm_fit --model_path=X.npy [--params_path=P.json] [--prior_type=Gaussian|Multinomial|Poisson]
//            [--gt_path=LABELS.npy] [--result_path=R.json] [--checkpoint_path=C.ckpt]
//            [--resume_path=C.ckpt] [--check_config]
//
// X.npy: N x d float32/float64 (Gaussian) or N x V integer counts
// (Multinomial, Poisson), C order.  P.json: the configuration object (keys as in
// paper_2204_08988_amd/fit.py: prior_type, alpha, iterations, burn_out,
// seed, k_max, precision, merge_form, hyper_params, learned, train_*).  The
// result JSON holds the labels, the weights, the NMI against the ground
// truth when given, the time per iteration and the K / log-posterior trace.
// --check_config parses the configuration and the data header, prints the
// resolved configuration as JSON and exits without touching a device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/dpmm.h"

namespace {

// ---------------------------------------------------------------- JSON values
struct Json {
  enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
  bool b = false;
  double num = 0.0;
  std::string str;
  std::vector<Json> arr;
  std::map<std::string, Json> obj;
  const Json* get(const std::string& k) const {
    if (kind != OBJ) return nullptr;
    auto it = obj.find(k);
    return it == obj.end() ? nullptr : &it->second;
  }
};

struct Parser {
  const std::string& s;
  size_t i = 0;
  explicit Parser(const std::string& text) : s(text) {}
  [[noreturn]] void fail(const std::string& what) {
    throw std::runtime_error("JSON: " + what + " at offset " + std::to_string(i));
  }
  void ws() {
    while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\t' || s[i] == '\r')) ++i;
  }
  bool lit(const char* w) {
    const size_t n = std::strlen(w);
    if (s.compare(i, n, w) == 0) {
      i += n;
      return true;
    }
    return false;
  }
  std::string string() {
    if (s[i] != '"') fail("string expected");
    ++i;
    std::string out;
    while (i < s.size() && s[i] != '"') {
      char c = s[i++];
      if (c == '\\') {
        if (i >= s.size()) fail("bad escape");
        const char e = s[i++];
        switch (e) {
          case 'n': c = '\n'; break;
          case 't': c = '\t'; break;
          case 'r': c = '\r'; break;
          case 'b': c = '\b'; break;
          case 'f': c = '\f'; break;
          case 'u': fail("\\u escapes are not supported");
          default: c = e;
        }
      }
      out.push_back(c);
    }
    if (i >= s.size()) fail("unterminated string");
    ++i;
    return out;
  }
  Json value() {
    ws();
    if (i >= s.size()) fail("value expected");
    Json v;
    const char c = s[i];
    if (c == '{') {
      v.kind = Json::OBJ;
      ++i;
      ws();
      if (s[i] == '}') {
        ++i;
        return v;
      }
      for (;;) {
        ws();
        std::string k = string();
        ws();
        if (s[i] != ':') fail("':' expected");
        ++i;
        v.obj[k] = value();
        ws();
        if (s[i] == ',') {
          ++i;
          continue;
        }
        if (s[i] == '}') {
          ++i;
          return v;
        }
        fail("',' or '}' expected");
      }
    }
    if (c == '[') {
      v.kind = Json::ARR;
      ++i;
      ws();
      if (s[i] == ']') {
        ++i;
        return v;
      }
      for (;;) {
        v.arr.push_back(value());
        ws();
        if (s[i] == ',') {
          ++i;
          continue;
        }
        if (s[i] == ']') {
          ++i;
          return v;
        }
        fail("',' or ']' expected");
      }
    }
    if (c == '"') {
      v.kind = Json::STR;
      v.str = string();
      return v;
    }
    if (lit("true")) {
      v.kind = Json::BOOL;
      v.b = true;
      return v;
    }
    if (lit("false")) {
      v.kind = Json::BOOL;
      return v;
    }
    if (lit("null")) return v;
    char* end = nullptr;
    v.num = std::strtod(s.c_str() + i, &end);
    if (end == s.c_str() + i) fail("number expected");
    v.kind = Json::NUM;
    i = (size_t)(end - s.c_str());
    return v;
  }
};

Json parse_json(const std::string& text) {
  Parser p(text);
  Json v = p.value();
  p.ws();
  if (p.i != text.size()) p.fail("trailing characters");
  return v;
}

std::string read_file(const std::string& path) {
  std::ifstream f(path, std::ios::binary);
  if (!f) throw std::runtime_error("cannot open " + path);
  std::stringstream ss;
  ss << f.rdbuf();
  return ss.str();
}

// ---------------------------------------------------------------- NPY arrays
struct Npy {
  std::string descr;             // '<f4', '<f8', '<i4', '<i8', ...
  std::vector<int64_t> shape;
  std::vector<char> data;
};

Npy read_npy(const std::string& path, bool header_only = false) {
  std::ifstream f(path, std::ios::binary);
  if (!f) throw std::runtime_error("cannot open " + path);
  char magic[8];
  f.read(magic, 8);
  if (!f || std::memcmp(magic, "\x93NUMPY", 6) != 0) throw std::runtime_error(path + " is not an .npy file");
  uint32_t hlen = 0;
  if (magic[6] == 1) {
    uint16_t h16 = 0;
    f.read(reinterpret_cast<char*>(&h16), 2);
    hlen = h16;
  } else {
    f.read(reinterpret_cast<char*>(&hlen), 4);
  }
  std::string h(hlen, ' ');
  f.read(&h[0], hlen);
  Npy a;
  auto field = [&](const char* key) {
    const size_t p = h.find(key);
    if (p == std::string::npos) throw std::runtime_error(path + ": header has no " + key);
    return h.substr(p + std::strlen(key));
  };
  std::string d = field("'descr':");
  const size_t q0 = d.find('\''), q1 = d.find('\'', q0 + 1);
  a.descr = d.substr(q0 + 1, q1 - q0 - 1);
  if (field("'fortran_order':").find("True") < 8) throw std::runtime_error(path + ": Fortran order is not supported");
  std::string sh = field("'shape':");
  sh = sh.substr(sh.find('(') + 1, sh.find(')') - sh.find('(') - 1);
  std::stringstream ss(sh);
  std::string tok;
  while (std::getline(ss, tok, ','))
    if (tok.find_first_not_of(' ') != std::string::npos) a.shape.push_back(std::stoll(tok));
  if (header_only) return a;
  int64_t count = 1;
  for (int64_t v : a.shape) count *= v;
  const int64_t item = std::stoll(a.descr.substr(2));
  if (a.descr[0] == '>') throw std::runtime_error(path + ": big-endian data is not supported");
  a.data.resize((size_t)(count * item));
  f.read(a.data.data(), (std::streamsize)a.data.size());
  if (!f) throw std::runtime_error(path + " is truncated");
  return a;
}

template <typename T>
std::vector<T> npy_as(const Npy& a) {
  int64_t count = 1;
  for (int64_t v : a.shape) count *= v;
  std::vector<T> out((size_t)count);
  const char kind = a.descr[1];
  const int item = std::stoi(a.descr.substr(2));
  for (int64_t j = 0; j < count; ++j) {
    const char* p = a.data.data() + j * item;
    double v = 0.0;
    if (kind == 'f' && item == 4) v = *reinterpret_cast<const float*>(p);
    else if (kind == 'f' && item == 8) v = *reinterpret_cast<const double*>(p);
    else if ((kind == 'i' || kind == 'u') && item == 4) v = kind == 'i' ? *reinterpret_cast<const int32_t*>(p)
                                                                           : *reinterpret_cast<const uint32_t*>(p);
    else if ((kind == 'i' || kind == 'u') && item == 8) v = (double)(kind == 'i' ? *reinterpret_cast<const int64_t*>(p)
                                                                                 : (int64_t)*reinterpret_cast<const uint64_t*>(p));
    else if ((kind == 'i' || kind == 'u') && item == 1) v = kind == 'i' ? *reinterpret_cast<const int8_t*>(p)
                                                                           : *reinterpret_cast<const uint8_t*>(p);
    else throw std::runtime_error("unsupported .npy dtype " + a.descr);
    out[(size_t)j] = (T)v;
  }
  return out;
}

// ---------------------------------------------------------------- configuration
struct Config {
  std::string prior_type = "Gaussian";
  double alpha = 10.0;
  int iterations = 100, burn_out = 15, k_max = 512, learned = 0;
  uint64_t seed = 1;
  std::string precision = "fp32", merge_form = "paper";
  int train_every = 10, train_until = 60, train_steps = 20, train_batch = 4096;
  double train_lr = 1e-3;
  double kappa = 1.0, nu = -1.0;
  std::vector<double> m, psi, beta, shape, rate;  // empty: data mean, identity, ones
};

Config parse_config(const Json& j, const std::string& prior_override) {
  Config c;
  if (j.kind != Json::OBJ && j.kind != Json::NUL) throw std::runtime_error("the configuration must be a JSON object");
  static const char* known[] = {"prior_type", "alpha", "iterations", "burn_out", "seed", "k_max", "precision",
                                "merge_form", "hyper_params", "learned", "train_every", "train_until", "train_steps",
                                "train_batch", "train_lr"};
  for (const auto& kv : j.obj) {
    bool ok = false;
    for (const char* k : known) ok = ok || kv.first == k;
    if (!ok) throw std::runtime_error("unknown configuration key " + kv.first);
  }
  auto num = [&](const char* k, double def) {
    const Json* v = j.get(k);
    if (!v) return def;
    if (v->kind != Json::NUM) throw std::runtime_error(std::string(k) + " must be a number");
    return v->num;
  };
  auto str = [&](const char* k, const std::string& def) {
    const Json* v = j.get(k);
    if (!v) return def;
    if (v->kind != Json::STR) throw std::runtime_error(std::string(k) + " must be a string");
    return v->str;
  };
  c.prior_type = prior_override.empty() ? str("prior_type", c.prior_type) : prior_override;
  if (c.prior_type != "Gaussian" && c.prior_type != "Multinomial" && c.prior_type != "Poisson")
    throw std::runtime_error("prior_type must be Gaussian, Multinomial or Poisson");
  c.alpha = num("alpha", c.alpha);
  c.iterations = (int)num("iterations", c.iterations);
  c.burn_out = (int)num("burn_out", c.burn_out);
  c.seed = (uint64_t)num("seed", (double)c.seed);
  c.k_max = (int)num("k_max", c.k_max);
  c.learned = (int)num("learned", c.learned);
  c.precision = str("precision", c.precision);
  c.merge_form = str("merge_form", c.merge_form);
  c.train_every = (int)num("train_every", c.train_every);
  c.train_until = (int)num("train_until", c.train_until);
  c.train_steps = (int)num("train_steps", c.train_steps);
  c.train_batch = (int)num("train_batch", c.train_batch);
  c.train_lr = num("train_lr", c.train_lr);
  if (const Json* hp = j.get("hyper_params")) {
    auto vec = [](const Json& a, std::vector<double>& out) {
      if (a.kind != Json::ARR) throw std::runtime_error("hyper_params arrays must be JSON arrays");
      for (const Json& e : a.arr) {
        if (e.kind == Json::ARR) {
          for (const Json& f : e.arr) out.push_back(f.num);
        } else {
          out.push_back(e.num);
        }
      }
    };
    if (const Json* v = hp->get("kappa")) c.kappa = v->num;
    if (const Json* v = hp->get("nu")) c.nu = v->num;
    if (const Json* v = hp->get("m")) vec(*v, c.m);
    if (const Json* v = hp->get("psi")) vec(*v, c.psi);
    if (const Json* v = hp->get("alpha")) vec(*v, c.beta);
    if (const Json* v = hp->get("shape")) vec(*v, c.shape);
    if (const Json* v = hp->get("rate")) vec(*v, c.rate);
  }
  return c;
}

std::string config_json(const Config& c, int64_t n, int d) {
  std::ostringstream o;
  o.precision(17);
  o << "{\"prior_type\": \"" << c.prior_type << "\", \"alpha\": " << c.alpha << ", \"iterations\": " << c.iterations
    << ", \"burn_out\": " << c.burn_out << ", \"seed\": " << c.seed << ", \"k_max\": " << c.k_max
    << ", \"precision\": \"" << c.precision << "\", \"merge_form\": \"" << c.merge_form
    << "\", \"learned\": " << c.learned << ", \"n\": " << n << ", \"d\": " << d << "}";
  return o.str();
}

#define HIPCHECK(e)                                                                                \
  do {                                                                                             \
    hipError_t _e = (e);                                                                           \
    if (_e != hipSuccess) throw std::runtime_error(std::string("HIP: ") + hipGetErrorString(_e)); \
  } while (0)

void check(dpmm_ctx* ctx, dpmm_status s, const char* what) {
  if (s != DPMM_OK)
    throw std::runtime_error(std::string(what) + ": " + dpmm_status_string(s) + ": " + dpmm_last_error(ctx));
}

int run(int argc, char** argv) {
  std::map<std::string, std::string> arg;
  for (int i = 1; i < argc; ++i) {
    std::string a = argv[i];
    if (a.rfind("--", 0) != 0) throw std::runtime_error("unexpected argument " + a);
    const size_t eq = a.find('=');
    arg[a.substr(2, eq == std::string::npos ? std::string::npos : eq - 2)] =
        eq == std::string::npos ? "1" : a.substr(eq + 1);
  }
  if (!arg.count("model_path")) throw std::runtime_error("--model_path=<data .npy> is required");
  Json cj;
  if (arg.count("params_path")) cj = parse_json(read_file(arg["params_path"]));
  std::string prior = arg.count("prior_type") ? arg["prior_type"] : "";
  if (!prior.empty() && prior.front() == '"') prior = prior.substr(1, prior.size() - 2);
  const Config c = parse_config(cj, prior);
  const bool gauss = c.prior_type == "Gaussian";
  Npy xa = read_npy(arg["model_path"], arg.count("check_config") > 0);
  if (xa.shape.size() != 2) throw std::runtime_error("the data must be a 2-d array");
  const int64_t n = xa.shape[0];
  const int d = (int)xa.shape[1];
  if (arg.count("check_config")) {
    std::printf("%s\n", config_json(c, n, d).c_str());
    return 0;
  }
  // host data
  std::vector<float> xf;
  std::vector<int32_t> xi;
  if (gauss)
    xf = npy_as<float>(xa);
  else
    xi = npy_as<int32_t>(xa);
  xa.data.clear();
  const bool pois = c.prior_type == "Poisson";
  std::vector<double> m = c.m, psi = c.psi, beta = c.beta, shape = c.shape, rate = c.rate;
  if (gauss) {
    if (m.empty()) {
      m.assign(d, 0.0);
      for (int64_t i = 0; i < n; ++i)
        for (int j = 0; j < d; ++j) m[j] += xf[(size_t)i * d + j];
      for (double& v : m) v /= (double)std::max<int64_t>(n, 1);
    }
    if (psi.empty()) {
      psi.assign((size_t)d * d, 0.0);
      for (int j = 0; j < d; ++j) psi[(size_t)j * d + j] = 1.0;
    }
    if ((int)m.size() != d || (int)psi.size() != d * d) throw std::runtime_error("hyper_params m / psi sizes");
  } else if (pois) {
    if (shape.empty()) shape.assign(d, 1.0);
    if (rate.empty()) rate.assign(d, 1.0);
    if ((int)shape.size() != d || (int)rate.size() != d) throw std::runtime_error("hyper_params shape / rate sizes");
  } else {
    if (beta.empty()) beta.assign(d, 1.0);
    if ((int)beta.size() != d) throw std::runtime_error("hyper_params alpha (Dirichlet) size");
  }
  dpmm_config cfg{};
  cfg.family = gauss ? DPMM_GAUSSIAN : (pois ? DPMM_POISSON : DPMM_MULTINOMIAL);
  cfg.d = d;
  cfg.k_max = c.k_max;
  cfg.burn_out = c.burn_out;
  cfg.alpha = c.alpha;
  cfg.kappa = c.kappa;
  cfg.nu = c.nu > 0 ? c.nu : d + 3.0;
  cfg.m = gauss ? m.data() : nullptr;
  cfg.psi = gauss ? psi.data() : nullptr;
  cfg.beta = gauss || pois ? nullptr : beta.data();
  cfg.gamma_shape = pois ? shape.data() : nullptr;
  cfg.gamma_rate = pois ? rate.data() : nullptr;
  cfg.seed = c.seed;
  cfg.precision = c.precision == "bf16" ? DPMM_BF16 : (c.precision == "bf16x3" ? DPMM_BF16X3 : DPMM_FP32);
  cfg.merge_form = c.merge_form == "inverse_split" ? DPMM_MERGE_INVERSE_SPLIT : DPMM_MERGE_PAPER;
  cfg.learned = c.learned;
  hipStream_t stream;
  HIPCHECK(hipStreamCreate(&stream));
  dpmm_ctx* ctx = nullptr;
  check(nullptr, dpmm_create(&cfg, stream, &ctx), "dpmm_create");
  std::unique_ptr<dpmm_ctx, void (*)(dpmm_ctx*)> guard(ctx, dpmm_destroy);
  void* dx = nullptr;
  int32_t* dz = nullptr;
  uint8_t* dzs = nullptr;
  const size_t xbytes = (size_t)n * d * 4;
  HIPCHECK(hipMalloc(&dx, std::max<size_t>(xbytes, 4)));
  HIPCHECK(hipMalloc((void**)&dz, std::max<size_t>((size_t)n * 4, 4)));
  HIPCHECK(hipMalloc((void**)&dzs, std::max<size_t>((size_t)n, 4)));
  HIPCHECK(hipMemcpy(dx, gauss ? (const void*)xf.data() : (const void*)xi.data(), xbytes, hipMemcpyHostToDevice));
  uint32_t t_done = 0;
  if (arg.count("resume_path"))
    check(ctx, dpmm_load_checkpoint(ctx, arg["resume_path"].c_str(), n, &t_done, dz, dzs), "dpmm_load_checkpoint");
  else
    check(ctx, dpmm_init_labels(ctx, n, dz, dzs), "dpmm_init_labels");
  dpmm_fit_options opt{};
  opt.t0 = t_done + 1;
  opt.iters = c.iterations;
  opt.train_every = c.learned ? c.train_every : 0;
  opt.train_until = c.train_until;
  opt.train_steps = c.train_steps;
  opt.train_batch = c.train_batch;
  opt.train_lr = (float)c.train_lr;
  std::vector<dpmm_iter_info> trace(std::max(c.iterations, 1));
  std::vector<double> secs(std::max(c.iterations, 1));
  check(ctx, dpmm_fit(ctx, dx, n, &opt, dz, dzs, trace.data(), secs.data()), "dpmm_fit");
  const uint32_t t_last = t_done + (uint32_t)c.iterations;
  if (arg.count("checkpoint_path"))
    check(ctx, dpmm_save_checkpoint(ctx, arg["checkpoint_path"].c_str(), n, t_last, dz, dzs), "dpmm_save_checkpoint");
  check(ctx, dpmm_sample_params(ctx, t_last + 1), "dpmm_sample_params");
  int32_t K = 0;
  check(ctx, dpmm_get_state(ctx, &K, nullptr), "dpmm_get_state");
  const size_t P = gauss ? (size_t)d + (size_t)d * d : (size_t)d;
  std::vector<double> log_pi(K), log_pisub(2 * (size_t)K), comp((size_t)K * 3 * P);
  check(ctx, dpmm_get_params(ctx, log_pi.data(), log_pisub.data(), comp.data()), "dpmm_get_params");
  std::vector<int32_t> labels((size_t)n);
  HIPCHECK(hipMemcpy(labels.data(), dz, (size_t)n * 4, hipMemcpyDeviceToHost));
  double nmi = NAN;
  if (arg.count("gt_path")) {
    const Npy g = read_npy(arg["gt_path"]);
    const std::vector<int32_t> gt = npy_as<int32_t>(g);
    if ((int64_t)gt.size() != n) throw std::runtime_error("the ground truth has another length");
    check(nullptr, dpmm_nmi(gt.data(), labels.data(), n, &nmi), "dpmm_nmi");
  }
  hipFree(dx);
  hipFree(dz);
  hipFree(dzs);
  std::ostringstream o;
  o.precision(17);
  o << "{\"K\": " << K << ", \"last_iteration\": " << t_last << ", \"labels\": [";
  for (int64_t i = 0; i < n; ++i) o << (i ? ", " : "") << labels[(size_t)i];
  o << "], \"weights\": [";
  for (int k = 0; k < K; ++k) o << (k ? ", " : "") << std::exp(log_pi[k]);
  o << "], \"iter_time\": [";
  for (int j = 0; j < c.iterations; ++j) o << (j ? ", " : "") << secs[j];
  o << "], \"K_trace\": [";
  for (int j = 0; j < c.iterations; ++j) o << (j ? ", " : "") << trace[j].K;
  o << "], \"logpost_trace\": [";
  for (int j = 0; j < c.iterations; ++j) o << (j ? ", " : "") << trace[j].logpost;
  o << "]";
  if (!std::isnan(nmi)) o << ", \"nmi\": " << nmi;
  o << ", \"config\": " << config_json(c, n, d) << "}\n";
  if (arg.count("result_path")) {
    std::ofstream f(arg["result_path"]);
    if (!f) throw std::runtime_error("cannot write " + arg["result_path"]);
    f << o.str();
  } else {
    std::fputs(o.str().c_str(), stdout);
  }
  std::fprintf(stderr, "dpmm_fit: %d iterations, K = %d%s\n", c.iterations, K,
               std::isnan(nmi) ? "" : (", NMI = " + std::to_string(nmi)).c_str());
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  try {
    return run(argc, argv);
  } catch (const std::exception& e) {
    std::fprintf(stderr, "dpmm_fit: %s\n", e.what());
    return 1;
  }
}
