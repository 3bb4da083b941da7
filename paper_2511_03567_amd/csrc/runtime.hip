// Host runtime of the residual engine: plan loading, tensor views, contraction
// execution (index permutation + MFMA GEMM), DF-chunked integrals, the
// particle-particle ladder, and the C ABI declared in include/ricmrcc.h.
#include <hip/hip_runtime.h>
#include <dlfcn.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <sstream>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include <rocsolver/rocsolver.h>

#include "../../include/ricmrcc.h"
#include "gemm.h"
#include "kernels.h"

namespace {

using ric::GemmArgs;
using ric::Iter;
using ric::kMaxDims;

// ---- ranges ---------------------------------------------------------------------------
enum Rng { RC = 0, RA, RV, RH, RP, RG, RX, NRNG };

Rng rng_of(char c) {
  switch (c) {
    case 'C': return RC;
    case 'A': return RA;
    case 'V': return RV;
    case 'H': return RH;
    case 'P': return RP;
    case 'G': return RG;
    case 'X': return RX;
  }
  throw std::runtime_error(std::string("bad range letter ") + c);
}

struct Sizes {
  int nc = 0, na = 0, nv = 0, naux = 0;
  long ext(Rng r) const {
    switch (r) {
      case RC: return nc;
      case RA: return na;
      case RV: return nv;
      case RH: return nc + na;
      case RP: return na + nv;
      case RG: return nc + na + nv;
      case RX: return naux;
      default: return 0;
    }
  }
  // offset of sub-range s inside declared range d
  long off(Rng d, Rng s) const {
    if (d == s) return 0;
    if (d == RG) {
      if (s == RC || s == RH) return 0;
      if (s == RA || s == RP) return nc;
      if (s == RV) return nc + na;
    }
    if (d == RH) {
      if (s == RC) return 0;
      if (s == RA) return nc;
    }
    if (d == RP) {
      if (s == RA) return 0;
      if (s == RV) return na;
    }
    throw std::runtime_error("sub-range not inside declared range");
  }
};

struct Err : std::runtime_error {
  int code;
  Err(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      throw Err(e_ == hipErrorOutOfMemory ? RIC_E_OOM : RIC_E_HIP,                       \
                std::string(#x) + ": " + hipGetErrorString(e_));                         \
  } while (0)

// ---- plan -------------------------------------------------------------------------------
struct Opd {
  int slot = -1;
  std::vector<Rng> sub;
  std::vector<int> lab;
};

enum Kind {
  K_ZERO, K_ALLOC, K_FREE, K_CONTRACT, K_CONTRACT0, K_ADD, K_DFC, K_SYMM, K_LADDER, K_MASK, K_SYMHALF, K_LADDERGRAD,
  K_LOOP, K_ENDLOOP
};

struct Op {
  Kind kind;
  double alpha = 1.0;
  std::vector<Opd> o;
  int slot = -1, slot2 = -1, slot3 = -1;
  bool chunked = false;   // ALLOC/FREE/ZERO of the slot a LOOP chunks
  std::vector<Rng> decl;  // for ALLOC
  std::string text;       // the plan line (for RIC_PROFILE=2)
};

struct Slot {
  std::string name;
  std::vector<Rng> decl;
  double* ptr = nullptr;
  const float* ptr32 = nullptr;   // FP32 copy for the mixed path, same layout (or null)
};

struct View {
  double* p = nullptr;
  const float* p32 = nullptr;     // the same elements in the slot's FP32 copy, if it has one
  int nd = 0;
  long ext[kMaxDims];
  long str[kMaxDims];
  int lab[kMaxDims];
  int find(int l) const {
    for (int i = 0; i < nd; ++i)
      if (lab[i] == l) return i;
    return -1;
  }
  long size() const {
    long s = 1;
    for (int i = 0; i < nd; ++i) s *= ext[i];
    return s;
  }
};

double parse_frac(const std::string& s) {
  auto k = s.find('/');
  if (k == std::string::npos) return std::stod(s);
  return std::stod(s.substr(0, k)) / std::stod(s.substr(k + 1));
}

// ---- device memory ----------------------------------------------------------------------
struct DevBuf {
  double* p = nullptr;
  size_t n = 0;
  void ensure(size_t elems) {
    if (elems <= n) return;
    if (p) HIPCHK(hipFree(p));
    p = nullptr;
    n = 0;
    HIPCHK(hipMalloc(&p, std::max<size_t>(elems, 1) * sizeof(double)));
    n = elems;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

// caching allocator for plan intermediates: exact-size free lists
struct Pool {
  std::multimap<size_t, double*> free_;
  std::vector<std::pair<double*, size_t>> all_;
  double* get(size_t elems) {
    elems = std::max<size_t>(elems, 1);
    auto it = free_.find(elems);
    if (it != free_.end()) {
      double* p = it->second;
      free_.erase(it);
      return p;
    }
    double* p = nullptr;
    if (hipMalloc(&p, elems * sizeof(double)) != hipSuccess) {
      // out of device memory: give back the idle blocks of other sizes and try once more
      (void)hipGetLastError();
      release_idle();
      HIPCHK(hipMalloc(&p, elems * sizeof(double)));
    }
    all_.push_back({p, elems});
    return p;
  }
  // free the blocks no intermediate holds (the next ALLOC of their size allocates again)
  void release_idle() {
    (void)hipDeviceSynchronize();  // queued kernels may still read blocks returned to the pool
    for (auto& kv : free_) {
      (void)hipFree(kv.second);
      all_.erase(std::find_if(all_.begin(), all_.end(),
                              [&](const std::pair<double*, size_t>& a) { return a.first == kv.second; }));
    }
    free_.clear();
  }
  void put(double* p, size_t elems) { free_.insert({std::max<size_t>(elems, 1), p}); }
  void release() {
    for (auto& a : all_) (void)hipFree(a.first);
    all_.clear();
    free_.clear();
  }
};

}  // namespace

// Device memory of the allocation-free update (ric_update_noalloc): the partial sums of the
// norm's two-pass reduction followed by the result slot.  One copy per GPU, held from the first
// context created on that GPU until the process ends, shared by every context there.  Host code
// never passes `scratch` itself to a kernel (in host code it names a host-side stand-in): it uses
// the device address hipGetSymbolAddress returns for the current device, kept per device below.
constexpr size_t kNoAllocDoubles = 8192;   // 64 KiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_addr;   // device -> address of that device's copy of `scratch`

// Address of `scratch` on `device`, looked up once per device; the device must be current.
double* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) return it->second;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr)
    throw Err(RIC_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_addr[device] = static_cast<double*>(p);
  return static_cast<double*>(p);
}
}  // namespace

// fp64 elements of split-K partial tiles (2 GiB)
constexpr size_t kSplitScratch = 256UL * 1024 * 1024;

struct ric_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  Sizes sz;
  bool spaces = false, have_f = false, have_B = false, have_rdm = false;

  // plan
  std::vector<std::string> plan_lines;
  std::vector<Slot> slots;
  std::unordered_map<std::string, int> slot_of;
  std::map<std::string, std::vector<Op>> sections;  // residual(_lin, _quad), energy, adjoint_t, adjoint_theta, energy_grad
  std::map<const std::vector<Op>*, std::pair<size_t, size_t>> ladder_block;   // ALLOC TAU .. FREE TAU

  // owned device tensors
  DevBuf f, eps, B, BT, BT32, g1, g2, g3, ga, ea, l2, k2, l3, k3, I4, I3, IJ, IK, tau, Edev, red, e0;
  DevBuf scrA, scrB, scrC, scrC2, scrK, wbuf, wbuf2, lad32, dfa, dfb, dfz, lgx, lgt, lgb, xr1, xl;
  Pool pool;
  rocblas_handle solver = nullptr;  // created on first use (blockwise eigensolver)
  const double* sc_B = nullptr;     // rotated quantities handed to the loaders by ric_semicanonicalize
  std::vector<const double*> sc_g;
  int precision = RIC_FP64;
  double ladder_ms = 0.0, total_ms = 0.0;
  bool ladder_ran = false;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  double* noalloc = nullptr;  // this device's copy of `scratch` (set by ric_create)
  const double* Bp = nullptr;  // the loaded DF factors: the owned copy B, or the caller's array (borrowed)
  bool accumulate_theta = false;  // adjoint (f, B) parts added to dF, dB instead of overwriting them
  // elements of W' per ladder chunk: six c rows at 809 orbitals for the forward residual; the
  // adjoint sections, whose intermediates take most of the device, keep three
  static constexpr double kLadderBudgetForward = 2.8e9, kLadderBudgetAdjoint = 1.4e9;
  double ladder_budget = kLadderBudgetAdjoint;
  void use_ladder_budget(double b) {
    if (b < ladder_budget) {   // return the larger chunk buffers before sections that need the room
      wbuf.release();
      wbuf2.release();
    }
    ladder_budget = b;
  }

  ~ric_ctx() {
    for (DevBuf* b : {&f, &eps, &B, &BT, &BT32, &g1, &g2, &g3, &ga, &ea, &l2, &k2, &l3, &k3, &I4, &I3, &IJ, &IK,
                      &tau, &Edev, &red, &e0, &scrA, &scrB, &scrC, &scrC2, &scrK, &wbuf, &wbuf2, &lad32, &dfa, &dfb, &dfz, &lgx, &lgt, &lgb, &xr1, &xl,
                      &sh_t1, &sh_t2, &sh_b, &sh_i4, &sh_i3, &sh_ij, &sh_ik})
      b->release();
    pool.release();
    if (solver) (void)rocblas_destroy_handle(solver);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }

  // -- plan parsing ---------------------------------------------------------------------
  int slot(const std::string& name, const std::vector<Rng>* decl = nullptr) {
    auto it = slot_of.find(name);
    if (it != slot_of.end()) return it->second;
    Slot s;
    s.name = name;
    if (decl) s.decl = *decl;
    slots.push_back(s);
    slot_of[name] = (int)slots.size() - 1;
    return (int)slots.size() - 1;
  }

  Opd parse_opd(const std::string& tok, std::map<std::string, int>& labels) {
    auto a = tok.find(':');
    auto b = tok.find(':', a + 1);
    if (a == std::string::npos || b == std::string::npos) throw Err(RIC_E_PLAN, "bad operand " + tok);
    Opd o;
    o.slot = slot(tok.substr(0, a));
    for (char c : tok.substr(a + 1, b - a - 1)) o.sub.push_back(rng_of(c));
    std::string ls = tok.substr(b + 1);
    std::stringstream ss(ls);
    std::string item;
    while (std::getline(ss, item, ',')) {
      if (item.empty()) continue;
      auto it = labels.find(item);
      int id;
      if (it == labels.end()) {
        id = (int)labels.size();
        labels[item] = id;
      } else {
        id = it->second;
      }
      o.lab.push_back(id);
    }
    if (o.lab.size() != o.sub.size()) throw Err(RIC_E_PLAN, "label/range count mismatch in " + tok);
    return o;
  }

  void load_plan(const std::string& path) {
    std::ifstream in(path);
    if (!in) throw Err(RIC_E_PLAN, "cannot open plan " + path);
    auto decl = [](const char* s) {
      std::vector<Rng> v;
      for (; *s; ++s) v.push_back(rng_of(*s));
      return v;
    };
    struct D { const char* n; const char* r; };
    const D fixed[] = {{"f", "GG"},     {"B", "XGG"},    {"T1", "HP"},   {"T2", "HHPP"}, {"gA", "AA"},
                       {"eA", "AA"},    {"K2", "AAAA"},  {"K3", "AAAAAA"}, {"I4", "HHHH"}, {"I3", "HHHP"},
                       {"IJ", "HHPP"},  {"IK", "HPHP"},  {"R1", "HP"},   {"R2", "HHPP"}, {"TAU", "HHPP"},
                       {"E", ""},       {"XR1", "HP"},   {"XL", "HHPP"}, {"YL", "HHPP"}, {"dT1", "HP"},
                       {"dT2", "HHPP"}, {"dF", "GG"},    {"dB", "XGG"}};
    for (auto& d : fixed) {
      auto v = decl(d.r);
      slot(d.n, &v);
    }
    std::string line;
    std::vector<Op>* cur = nullptr;
    std::vector<size_t> loops;  // open LOOP operations of the current section
    int loop_slot = -1;
    while (std::getline(in, line)) {
      if (line.empty() || line[0] == '#') continue;
      std::stringstream ss(line);
      std::vector<std::string> t;
      std::string w;
      while (ss >> w) t.push_back(w);
      if (t.empty()) continue;
      if (t[0] == "SECTION") {
        cur = &sections[t.at(1)];
        continue;
      }
      if (t[0] == "END") {
        if (!loops.empty()) throw Err(RIC_E_PLAN, "LOOP without ENDLOOP");
        cur = nullptr;
        continue;
      }
      if (!cur) throw Err(RIC_E_PLAN, "operation outside a section: " + line);
      Op op;
      const bool in_loop = !loops.empty();
      std::map<std::string, int> labels;
      if (t[0] == "ALLOC") {
        op.kind = K_ALLOC;
        auto v = decl(t.at(2).c_str());
        op.slot = slot(t.at(1), &v);
        slots[op.slot].decl = v;
        op.decl = v;
      } else if (t[0] == "FREE") {
        op.kind = K_FREE;
        op.slot = slot(t.at(1));
      } else if (t[0] == "ZERO") {
        op.kind = K_ZERO;
        op.slot = slot(t.at(1));
      } else if (t[0] == "CONTRACT" || t[0] == "CONTRACT0") {
        op.kind = t[0] == "CONTRACT" ? K_CONTRACT : K_CONTRACT0;
        op.alpha = parse_frac(t.at(1));
        for (int i = 2; i < 5; ++i) op.o.push_back(parse_opd(t.at(i), labels));
      } else if (t[0] == "ADD") {
        op.kind = K_ADD;
        op.alpha = parse_frac(t.at(1));
        for (int i = 2; i < 4; ++i) op.o.push_back(parse_opd(t.at(i), labels));
      } else if (t[0] == "DFC") {
        op.kind = K_DFC;
        op.alpha = parse_frac(t.at(1));
        for (int i = 2; i < 6; ++i) op.o.push_back(parse_opd(t.at(i), labels));
      } else if (t[0] == "SYMMETRIZE") {
        op.kind = K_SYMM;
        op.slot = slot(t.at(1));
      } else if (t[0] == "SYMHALF") {
        op.kind = K_SYMHALF;
        op.slot = slot(t.at(1));
      } else if (t[0] == "LADDER") {
        op.kind = K_LADDER;  // LADDER out in: out += (ce|df) in
        op.slot = slot(t.at(1));
        op.slot2 = slot(t.at(2));
      } else if (t[0] == "LADDERGRAD") {
        op.kind = K_LADDERGRAD;  // LADDERGRAD dB x tau
        op.slot = slot(t.at(1));
        op.slot2 = slot(t.at(2));
        op.slot3 = slot(t.at(3));
      } else if (t[0] == "MASK") {
        op.kind = K_MASK;  // MASK singles doubles
        op.slot = slot(t.at(1));
        op.slot2 = slot(t.at(2));
      } else if (t[0] == "LOOP") {
        // LOOP name dim: the body runs once per chunk of dimension dim of intermediate name
        if (!loops.empty()) throw Err(RIC_E_PLAN, "nested LOOP");
        op.kind = K_LOOP;
        op.slot = slot(t.at(1));
        op.slot2 = std::stoi(t.at(2));
        if (op.slot2 != 0) throw Err(RIC_E_PLAN, "LOOP chunks the leading dimension only");
        loops.push_back(cur->size());
        loop_slot = op.slot;
      } else if (t[0] == "ENDLOOP") {
        if (loops.empty()) throw Err(RIC_E_PLAN, "ENDLOOP without LOOP");
        op.kind = K_ENDLOOP;
        (*cur)[loops.back()].slot3 = (int)cur->size();
        loops.pop_back();
        loop_slot = -1;
      } else {
        throw Err(RIC_E_PLAN, "unknown plan operation " + t[0]);
      }
      if (in_loop && op.slot == loop_slot && (op.kind == K_ALLOC || op.kind == K_FREE || op.kind == K_ZERO))
        op.chunked = true;
      if (op.kind == K_CONTRACT || op.kind == K_CONTRACT0 || op.kind == K_DFC) op.text = line;
      cur->push_back(op);
    }
    for (const char* need : {"residual", "residual_lin", "residual_quad", "energy", "adjoint_t", "adjoint_theta",
                             "energy_grad"})
      if (sections.find(need) == sections.end()) throw Err(RIC_E_PLAN, std::string("plan has no section ") + need);
    for (auto& kv : sections) {
      size_t b = kv.second.size(), e = kv.second.size();
      for (size_t i = 0; i < kv.second.size(); ++i) {
        const Op& op = kv.second[i];
        if (op.slot >= 0 && slots[op.slot].name == "TAU") {
          if (op.kind == K_ALLOC && b == kv.second.size()) b = i;
          if (op.kind == K_FREE) e = i;
        }
      }
      if (b < kv.second.size() && e < kv.second.size()) ladder_block[&kv.second] = {b, e};
    }
  }

  // -- views ------------------------------------------------------------------------------
  View view(const Opd& o) {
    const Slot& s = slots.at(o.slot);
    bool empty = false;
    for (Rng r : o.sub) empty = empty || sz.ext(r) == 0;
    if (!s.ptr && s.decl.size() > 0 && !empty) throw Err(RIC_E_STATE, "tensor " + s.name + " is not available");
    View v;
    v.nd = (int)o.sub.size();
    if (v.nd != (int)s.decl.size()) throw Err(RIC_E_PLAN, "rank mismatch for " + s.name);
    long stride = 1;
    long full[kMaxDims];
    for (int i = v.nd - 1; i >= 0; --i) {
      full[i] = stride;
      stride *= sz.ext(s.decl[i]);
    }
    long off = 0;
    for (int i = 0; i < v.nd; ++i) {
      v.ext[i] = sz.ext(o.sub[i]);
      v.str[i] = full[i];
      v.lab[i] = o.lab[i];
      off += sz.off(s.decl[i], o.sub[i]) * full[i];
    }
    v.p = empty ? nullptr : s.ptr + off;
    v.p32 = (empty || !s.ptr32) ? nullptr : s.ptr32 + off;
    return v;
  }

  // -- FP32 copies of stored operands for the mixed path ----------------------------------------
  // The amplitudes are copied at each mixed residual; the DF factors and the stored integral
  // blocks once after each ric_load_df.  Large FP32 products read these in place instead of
  // converting their operands product by product.
  DevBuf sh_t1, sh_t2, sh_b, sh_i4, sh_i3, sh_ij, sh_ik;
  bool shadows_static = false;

  // A copy is made only while at least kShadowReserve bytes of the device stay free; an operand
  // without one is converted product by product as before.
  static constexpr size_t kShadowReserve = 16UL << 30;

  void make_shadow(const char* name, DevBuf& buf) {
    const int id = slot_of.at(name);
    Slot& s = slots[id];
    s.ptr32 = nullptr;
    const long n = slot_elems(id);
    if (!s.ptr || n == 0) return;
    const size_t need = ((size_t)n + 1) / 2;
    if (buf.n < need) {
      size_t free_b = 0, total_b = 0;
      HIPCHK(hipMemGetInfo(&free_b, &total_b));
      if (free_b + buf.n * sizeof(double) < need * sizeof(double) + kShadowReserve) {
        buf.release();
        return;
      }
    }
    buf.ensure(need);
    View v;
    v.p = s.ptr;
    v.nd = (int)s.decl.size();
    long st = 1;
    for (int i = v.nd - 1; i >= 0; --i) {
      v.ext[i] = sz.ext(s.decl[i]);
      v.str[i] = st;
      v.lab[i] = i;
      st *= v.ext[i];
    }
    std::vector<int> ord(v.nd);
    for (int i = 0; i < v.nd; ++i) ord[i] = i;
    gather(v, ord, nullptr, reinterpret_cast<float*>(buf.p));
    s.ptr32 = reinterpret_cast<const float*>(buf.p);
  }

  void static_shadows() {
    if (shadows_static) return;
    make_shadow("IK", sh_ik);
    make_shadow("IJ", sh_ij);
    make_shadow("B", sh_b);
    make_shadow("I3", sh_i3);
    make_shadow("I4", sh_i4);
    shadows_static = true;
  }

  void drop_shadows() {
    for (const char* nm : {"B", "I4", "I3", "IJ", "IK", "T1", "T2"}) slots[slot_of.at(nm)].ptr32 = nullptr;
    for (DevBuf* b : {&sh_b, &sh_i4, &sh_i3, &sh_ij, &sh_ik, &sh_t1, &sh_t2}) b->release();
    shadows_static = false;
  }

  long slot_elems(int id) {
    long n = 1;
    for (Rng r : slots[id].decl) n *= sz.ext(r);
    return n;
  }

  // -- primitive: out[lab order] (beta) += alpha * in[perm] ------------------------------------
  void axpby(const View& out, double alpha, const View& in, double beta) {
    Iter it;
    it.nd = out.nd;
    it.total = 1;
    for (int i = 0; i < out.nd; ++i) {
      it.ext[i] = out.ext[i];
      it.so[i] = out.str[i];
      int j = in.find(out.lab[i]);
      if (j < 0) throw Err(RIC_E_PLAN, "ADD: label missing in input");
      it.si[i] = in.str[j];
      it.total *= out.ext[i];
    }
    if (in.nd != out.nd) throw Err(RIC_E_PLAN, "ADD: rank mismatch");
    if (it.nd == 0) it.total = 1;
    HIPCHK(ric::strided_copy(it, alpha, in.p, beta, out.p, stream));
  }

  // gather view dims in the given order into a contiguous buffer
  // dst[order] <- v; with nk > 0 the last nk dimensions of `order` form rows of length kp
  // (>= their product), the padding zero-filled
  void gather(const View& v, const std::vector<int>& order, double* dst, float* dst32, size_t nk = 0, long kp = 0) {
    Iter it;
    it.nd = (int)order.size();
    it.total = 1;
    long st = 1, total = 1;
    long kprod = 1;
    for (size_t i = order.size() - nk; i < order.size(); ++i) kprod *= v.ext[order[i]];
    const bool padded = nk > 0 && kp > kprod;
    for (int i = it.nd - 1; i >= 0; --i) {
      it.ext[i] = v.ext[order[i]];
      it.si[i] = v.str[order[i]];
      it.so[i] = st;
      st *= it.ext[i];
      total *= it.ext[i];
      if (padded && i == it.nd - (int)nk) st = kp;  // rows of the padded length
    }
    it.total = total;
    if (padded) {
      const long rows = kprod > 0 ? total / kprod : 0;
      if (dst32) HIPCHK(ric::fill(reinterpret_cast<double*>(dst32), (rows * kp + 1) / 2, 0.0, stream));
      else HIPCHK(ric::fill(dst, rows * kp, 0.0, stream));
    }
    if (dst32) HIPCHK(ric::strided_copy_f32(it, 1.0, v.p, dst32, stream));
    else HIPCHK(ric::strided_copy(it, 1.0, v.p, 0.0, dst, stream));
  }

  // dims (in order) mergeable into one index of stride `s` (product extent)?
  static bool mergeable(const View& v, const std::vector<int>& dims, long& s) {
    s = 1;
    if (dims.empty()) return true;
    long expect = -1;
    for (int i = (int)dims.size() - 1; i >= 0; --i) {
      const int d = dims[i];
      if (v.ext[d] == 1) continue;
      if (expect < 0) {
        s = v.str[d];
        expect = v.str[d] * v.ext[d];
      } else {
        if (v.str[d] != expect) return false;
        expect = v.str[d] * v.ext[d];
      }
    }
    return true;
  }

  // products above this many flops get K padded to the vector width (RIC_PAD_MIN_FLOPS overrides)
  double pad_min_flops = getenv("RIC_PAD_MIN_FLOPS") ? std::atof(getenv("RIC_PAD_MIN_FLOPS")) : 1e10;
  // in RIC_FP32MIX, products above this many flops take fp32 operands (RIC_FP32_MIN_FLOPS overrides)
  double fp32_min_flops = getenv("RIC_FP32_MIN_FLOPS") ? std::atof(getenv("RIC_FP32_MIN_FLOPS")) : 1e10;

  // -- contraction out (+)= alpha * sum a * b -------------------------------------------------
  void contract(const View& out, double alpha, const View& a0, const View& b0, bool fresh, bool allow32) {
    // C = A B^T is written row by row: the operand carrying the output's innermost index takes
    // the role of B, so the product lands in the output's own layout
    const View* pa = &a0;
    const View* pb = &b0;
    {
      int inner = -1;
      long best = -1;
      for (int i = 0; i < out.nd; ++i)
        if (out.ext[i] > 1 && (best < 0 || out.str[i] < best)) {
          best = out.str[i];
          inner = i;
        }
      if (inner >= 0 && a0.find(out.lab[inner]) >= 0 && b0.find(out.lab[inner]) < 0) std::swap(pa, pb);
    }
    const View& a = *pa;
    const View& b = *pb;
    std::vector<int> aM, aK, bN, bK, oM, oN;
    for (int i = 0; i < out.nd; ++i) {
      const int l = out.lab[i];
      const int ia = a.find(l), ib = b.find(l);
      if (ia >= 0 && ib >= 0) throw Err(RIC_E_PLAN, "batch labels are not supported");
      if (ia >= 0) {
        aM.push_back(ia);
        oM.push_back(i);
      } else if (ib >= 0) {
        bN.push_back(ib);
        oN.push_back(i);
      } else {
        throw Err(RIC_E_PLAN, "output label not in operands");
      }
    }
    for (int i = 0; i < a.nd; ++i) {
      const int l = a.lab[i];
      if (out.find(l) >= 0) continue;
      const int ib = b.find(l);
      if (ib < 0) throw Err(RIC_E_PLAN, "label summed in one operand only");
      aK.push_back(i);
      bK.push_back(ib);
    }
    for (int i = 0; i < b.nd; ++i)
      if (out.find(b.lab[i]) < 0 && a.find(b.lab[i]) < 0) throw Err(RIC_E_PLAN, "label summed in one operand only");
    long M = 1, N = 1, K = 1;
    for (int d : aM) M *= a.ext[d];
    for (int d : bN) N *= b.ext[d];
    for (int d : aK) K *= a.ext[d];
    if (M == 0 || N == 0) return;
    if (K == 0) {
      if (fresh) HIPCHK(ric::fill(out.p, out.size(), 0.0, stream));  // fresh outputs are contiguous
      return;
    }
    const double flops = 2.0 * (double)M * N * K;
    const bool use32 = allow32 && precision == RIC_FP32MIX && flops > fp32_min_flops;

    // energy-type full contraction: dot product
    if (M == 1 && N == 1 && !use32) {
      std::vector<int> ka = aK, kb = bK;
      const double* pa;
      const double* pb;
      long sa, sb;
      bool ca = mergeable(a, ka, sa) && sa == 1;
      bool cb = mergeable(b, kb, sb) && sb == 1;
      scrA.ensure(ca ? 0 : K);
      scrB.ensure(cb ? 0 : K);
      if (ca) pa = a.p; else { gather(a, ka, scrA.p, nullptr); pa = scrA.p; }
      if (cb) pb = b.p; else { gather(b, kb, scrB.p, nullptr); pb = scrB.p; }
      red.ensure(ric::kReducePartials);
      if (fresh) HIPCHK(ric::fill(out.p, 1, 0.0, stream));
      HIPCHK(ric::dot_accumulate(pa, pb, K, alpha, out.p, red.p, stream));
      return;
    }

    // operand A as [M][K], B as [N][K]
    std::vector<int> ordA = aM, ordB = bN;
    ordA.insert(ordA.end(), aK.begin(), aK.end());
    ordB.insert(ordB.end(), bK.begin(), bK.end());
    long sAm, sAk, sBn, sBk;
    // in mixed precision an operand is read in place only from its FP32 copy
    const bool inA = !use32 || a.p32 != nullptr, inB = !use32 || b.p32 != nullptr;
    bool directA = inA && mergeable(a, aM, sAm) && mergeable(a, aK, sAk) && sAk == 1;
    bool directB = inB && mergeable(b, bN, sBn) && mergeable(b, bK, sBk) && sBk == 1;
    if (directA && M > 1 && sAm < K) directA = false;
    if (directB && N > 1 && sBn < K) directB = false;
    if (M == 1) sAm = K;
    if (N == 1) sBn = K;
    // otherwise an operand whose M (N) indices are contiguous and K indices strided is read
    // K-major in place
    bool tA = false, tB = false;
    long tldA = 0, tldB = 0;
    if (inA && !directA && M > 1 && K > 1) {
      long sm, sk;
      if (mergeable(a, aM, sm) && sm == 1 && mergeable(a, aK, sk) && sk >= M) {
        tA = true;
        tldA = sk;
      }
    }
    if (inB && !directB && N > 1 && K > 1) {
      long sn, sk;
      if (mergeable(b, bN, sn) && sn == 1 && mergeable(b, bK, sk) && sk >= N) {
        tB = true;
        tldB = sk;
      }
    }
    // output as [M][N]
    long sOm, sOn;
    bool directC = mergeable(out, oM, sOm) && mergeable(out, oN, sOn) && (sOn == 1 || N == 1);
    if (directC && M > 1 && N > 1 && sOm < N) directC = false;
    if (M == 1) sOm = N;

    // K not a multiple of the GEMM's vector width (2 doubles / 4 floats): for large products
    // both operands are gathered into rows of Kp >= K with zero padding so the 16-byte load
    // path applies (the padding adds zero terms).  Skinny products (an output side of at
    // most 16) are bound by reading the large operand once: they read it in place with
    // scalar loads rather than copy it.
    const long vw = use32 ? 4 : 2;
    const bool skinny = !use32 && std::min(M, N) <= 16;
    long Kp = K;
    if (K % vw != 0 && flops > pad_min_flops && !aK.empty() && !skinny) {
      Kp = (K + vw - 1) / vw * vw;
      directA = directB = tA = tB = false;
    }
    // large products keep 16-byte loads: a K-major operand needs its contiguous extent and
    // leading dimension in whole vectors, else it is gathered
    if (flops > pad_min_flops && !skinny) {
      if (tA && (M % vw != 0 || tldA % vw != 0)) tA = false;
      if (tB && (N % vw != 0 || tldB % vw != 0)) tB = false;
    }
    if (!directA && !tA) scrA.ensure(use32 ? ((size_t)M * Kp + 1) / 2 : (size_t)M * Kp);
    if (!directB && !tB) scrB.ensure(use32 ? ((size_t)N * Kp + 1) / 2 : (size_t)N * Kp);
    const double* pA = use32 ? reinterpret_cast<const double*>(a.p32) : a.p;
    const double* pB = use32 ? reinterpret_cast<const double*>(b.p32) : b.p;
    if (tA) sAm = tldA;
    if (tB) sBn = tldB;
    if (!directA && !tA) {
      gather(a, ordA, use32 ? nullptr : scrA.p, use32 ? reinterpret_cast<float*>(scrA.p) : nullptr, aK.size(), Kp);
      pA = scrA.p;
      sAm = Kp;
    }
    if (!directB && !tB) {
      gather(b, ordB, use32 ? nullptr : scrB.p, use32 ? reinterpret_cast<float*>(scrB.p) : nullptr, bK.size(), Kp);
      pB = scrB.p;
      sBn = Kp;
    }
    GemmArgs g;
    g.ta = tA;
    g.tb = tB;
    g.M = (int)M;
    g.N = (int)N;
    g.K = (int)Kp;
    if (M > 2147483647L || N > 2147483647L || Kp > 2147483647L) throw Err(RIC_E_ARG, "contraction too large");
    g.lda = sAm;
    g.ldb = sBn;
    scrK.ensure(kSplitScratch);
    if (directC) {
      g.alpha = alpha;
      g.beta = fresh ? 0.0 : 1.0;
      g.C = out.p;
      g.ldc = sOm;
    } else {
      scrC.ensure((size_t)M * N);
      g.alpha = 1.0;
      g.beta = 0.0;
      g.C = scrC.p;
      g.ldc = N;
    }
    if (use32)
      HIPCHK(ric::gemm_nt_f32(g, reinterpret_cast<const float*>(pA), reinterpret_cast<const float*>(pB), stream,
                              scrK.p, scrK.n));
    else
      HIPCHK(ric::gemm_nt_f64(g, pA, pB, stream, scrK.p, scrK.n));
    if (!directC) {
      // out[dims] (+)= alpha * Ctmp[M][N]
      Iter it;
      it.nd = out.nd;
      it.total = 1;
      long stM[kMaxDims], stN[kMaxDims];
      {
        long s = N;
        for (int i = (int)oM.size() - 1; i >= 0; --i) { stM[i] = s; s *= out.ext[oM[i]]; }
        s = 1;
        for (int i = (int)oN.size() - 1; i >= 0; --i) { stN[i] = s; s *= out.ext[oN[i]]; }
      }
      for (int i = 0; i < out.nd; ++i) {
        it.ext[i] = out.ext[i];
        it.so[i] = out.str[i];
        it.total *= out.ext[i];
        auto pm = std::find(oM.begin(), oM.end(), i);
        if (pm != oM.end()) it.si[i] = stM[pm - oM.begin()];
        else it.si[i] = stN[std::find(oN.begin(), oN.end(), i) - oN.begin()];
      }
      HIPCHK(ric::strided_copy(it, alpha, scrC.p, fresh ? 0.0 : 1.0, out.p, stream));
    }
  }

  // -- (pr|qs) = sum_X L1[X,p,r] L2[X,q,s] built block by block and contracted with y ---------
  // Product of the extents of the distinct labels of `vs` (label X of the DF factors excluded
  // when skip >= 0).
  static double label_volume(std::initializer_list<const View*> vs, int skip) {
    std::map<int, long> ex;
    for (const View* v : vs)
      for (int i = 0; i < v->nd; ++i) ex[v->lab[i]] = v->ext[i];
    double p = 1.0;
    for (auto& kv : ex)
      if (kv.first != skip) p *= (double)kv.second;
    return p;
  }

  // out += alpha * sum (pr|qs) y without forming (pr|qs): Z = Lb . y over the labels of Lb that
  // y holds and neither out nor La does, then out += alpha * La . Z (sum over X and the labels
  // La shares with Z).  Returns false when a label would have to be carried through both
  // products (a batch label).  With dry = true only the flops and the size of Z are reported.
  bool dfc_through_factors(const View& out, double alpha, const View& La, const View& Lb, const View& y, bool dry,
                           double& flops, double& zsize) {
    const int xl = Lb.lab[0];
    std::vector<int> zl{xl};
    std::vector<long> ze{Lb.ext[0]};
    for (int i = 1; i < Lb.nd; ++i) {
      const int l = Lb.lab[i];
      const bool summed = y.find(l) >= 0 && out.find(l) < 0 && La.find(l) < 0;
      if (summed) continue;
      if (y.find(l) >= 0) return false;
      zl.push_back(l);
      ze.push_back(Lb.ext[i]);
    }
    for (int i = 0; i < y.nd; ++i) {
      if (Lb.find(y.lab[i]) >= 0) continue;
      zl.push_back(y.lab[i]);
      ze.push_back(y.ext[i]);
    }
    if ((int)zl.size() > kMaxDims) return false;
    for (size_t i = 1; i < zl.size(); ++i)
      if (La.find(zl[i]) >= 0 && out.find(zl[i]) >= 0) return false;
    for (int i = 0; i < out.nd; ++i)
      if (La.find(out.lab[i]) < 0 && std::find(zl.begin(), zl.end(), out.lab[i]) == zl.end()) return false;
    View z;
    z.nd = (int)zl.size();
    long st = 1;
    for (int i = z.nd - 1; i >= 0; --i) {
      z.lab[i] = zl[i];
      z.ext[i] = ze[i];
      z.str[i] = st;
      st *= ze[i];
    }
    const double nx = (double)Lb.ext[0];
    flops = 2.0 * nx * label_volume({&Lb, &y}, xl) + 2.0 * nx * label_volume({&La, &z}, xl);
    zsize = (double)st;
    if (dry) return true;
    dfz.ensure((size_t)std::max<long>(st, 1));
    z.p = dfz.p;
    contract(z, 1.0, Lb, y, true, true);
    contract(out, alpha, La, z, false, true);
    return true;
  }

  void dfc(const View& out, double alpha, const View& L1, const View& L2, const View& y) {
    const long np_ = L1.ext[1], nr = L1.ext[2], nq = L2.ext[1], ns = L2.ext[2], nx = L1.ext[0];
    if (np_ == 0 || nr == 0 || nq == 0 || ns == 0) return;
    {
      // the cheaper of building the integral block and going through the factors
      View e;
      e.nd = 4;
      const int lb4[4] = {L1.lab[1], L1.lab[2], L2.lab[1], L2.lab[2]};
      const long ex4[4] = {np_, nr, nq, ns};
      for (int i = 0; i < 4; ++i) {
        e.lab[i] = lb4[i];
        e.ext[i] = ex4[i];
      }
      const double build = 2.0 * (double)nx * np_ * nr * nq * ns + 2.0 * label_volume({&e, &y, &out}, -1);
      double f1 = 0, z1 = 0, f2 = 0, z2 = 0;
      const double zmax = 2.0e9;
      bool ok1 = dfc_through_factors(out, alpha, L1, L2, y, true, f1, z1) && z1 <= zmax;
      bool ok2 = dfc_through_factors(out, alpha, L2, L1, y, true, f2, z2) && z2 <= zmax;
      if (ok1 && (!ok2 || f1 <= f2) && f1 < build) {
        dfc_through_factors(out, alpha, L1, L2, y, false, f1, z1);
        return;
      }
      if (ok2 && f2 < build) {
        dfc_through_factors(out, alpha, L2, L1, y, false, f2, z2);
        return;
      }
    }
    // L2 as [(q,s)][X]; in mixed precision the block is built from FP32 copies of the factors
    // (FP32 tiles, FP64 carry per K slab, FP64 block) like the other large products
    const bool use32 = precision == RIC_FP32MIX && 2.0 * (double)nx * np_ * nr * nq * ns > fp32_min_flops;
    DevBuf& l2buf = dfb;
    l2buf.ensure(use32 ? ((size_t)nq * ns * nx + 1) / 2 : (size_t)nq * ns * nx);
    gather(L2, {1, 2, 0}, use32 ? nullptr : l2buf.p, use32 ? reinterpret_cast<float*>(l2buf.p) : nullptr);
    const long per = std::max<long>(1, (long)(1.2e9 / std::max<long>(1, nr * nq * ns)));
    const long chunk = std::min(np_, per);
    const int lp = L1.lab[1];
    for (long p0 = 0; p0 < np_; p0 += chunk) {
      const long pc = std::min(chunk, np_ - p0);
      View l1c = L1;
      l1c.p += p0 * L1.str[1];
      l1c.ext[1] = pc;
      dfa.ensure(use32 ? ((size_t)pc * nr * nx + 1) / 2 : (size_t)pc * nr * nx);
      gather(l1c, {1, 2, 0}, use32 ? nullptr : dfa.p, use32 ? reinterpret_cast<float*>(dfa.p) : nullptr);
      wbuf.ensure((size_t)pc * nr * nq * ns);
      GemmArgs g;
      g.M = (int)(pc * nr);
      g.N = (int)(nq * ns);
      g.K = (int)nx;
      g.lda = nx;
      g.ldb = nx;
      g.C = wbuf.p;
      g.ldc = nq * ns;
      scrK.ensure(kSplitScratch);
      if (use32)
        HIPCHK(ric::gemm_nt_f32(g, reinterpret_cast<const float*>(dfa.p), reinterpret_cast<const float*>(l2buf.p),
                                stream, scrK.p, scrK.n));
      else
        HIPCHK(ric::gemm_nt_f64(g, dfa.p, l2buf.p, stream, scrK.p, scrK.n));
      View e;
      e.p = wbuf.p;
      e.nd = 4;
      const long ex[4] = {pc, nr, nq, ns};
      const int lb[4] = {lp, L1.lab[2], L2.lab[1], L2.lab[2]};
      long st = 1;
      for (int i = 3; i >= 0; --i) {
        e.ext[i] = ex[i];
        e.str[i] = st;
        e.lab[i] = lb[i];
        st *= ex[i];
      }
      View oc = out, yc = y;
      for (View* v : {&oc, &yc}) {
        int d = v->find(lp);
        if (d >= 0) {
          v->p += p0 * v->str[d];
          v->ext[d] = pc;
        }
      }
      contract_keep_scratch(oc, alpha, e, yc);
    }
  }

  // contraction whose operand `e` lives in wbuf and must not be overwritten by gathers
  void contract_keep_scratch(const View& out, double alpha, const View& e, const View& y) {
    // e is contiguous; the contraction only gathers into scrA/scrB/scrC, never wbuf
    contract(out, alpha, e, y, false, true);
  }

  // -- ladder: R2[k,l,c,d] += sum_{e,f} (ce|df) tau[k,l,e,f] ------------------------------------
  // With tau pair-symmetric, only c >= d is built: W[c,d,e,f] = (ce|df) from B in chunks of c,
  // packed to W+/- over e >= f (e > f) and contracted with tau+/- over k <= l (k < l):
  // R2[k,l,c,d] = S+[kl,cd] + S-[kl,cd], R2[l,k,c,d] = S+ - S-, R2[l,k,d,c] = R2[k,l,c,d].
  void ladder(const double* taup, double* r2) {
    const int np_ = sz.na + sz.nv, nh = sz.nc + sz.na, nx = sz.naux;
    if (np_ == 0 || nh == 0) return;
    const long pp = (long)np_ * np_;
    const long nhp = (long)nh * (nh + 1) / 2, nhm = (long)nh * (nh - 1) / 2;
    const long npp = (long)np_ * (np_ + 1) / 2, npm = (long)np_ * (np_ - 1) / 2;
    const long ldp = (npp + 3) / 4 * 4, ldm = std::max<long>(4, (npm + 3) / 4 * 4);
    const bool mixed = precision == RIC_FP32MIX;
    if (BT.n < (size_t)pp * nx) throw Err(RIC_E_STATE, "DF factors not loaded");
    // packed tau (fp64, or fp32 for the mixed path)
    const size_t tel = (size_t)nhp * ldp + (size_t)nhm * ldm;
    lad32.ensure(mixed ? (tel + 1) / 2 : tel);
    double* tpd = lad32.p;
    double* tmd = lad32.p + (size_t)nhp * ldp;
    float* tpf = reinterpret_cast<float*>(lad32.p);
    float* tmf = tpf + (size_t)nhp * ldp;
    if (mixed) HIPCHK(ric::pack_tau_f32(taup, nh, np_, tpf, tmf, ldp, ldm, stream));
    else HIPCHK(ric::pack_tau(taup, nh, np_, tpd, tmd, ldp, ldm, stream));
    // chunk of c rows: W'[(c,e)][(d,f)] (one GEMM), then W+/- per (c,d) pair
    // elements of W' per chunk (RIC_LADDER_BUDGET overrides)
    const double budget = getenv("RIC_LADDER_BUDGET") ? std::atof(getenv("RIC_LADDER_BUDGET")) : ladder_budget;
    long chunk = std::max<long>(1, (long)(budget / ((double)np_ * pp)));
    chunk = std::min<long>(chunk, np_);
    const size_t wel = (size_t)chunk * np_ * pp;
    const size_t pel = (size_t)chunk * np_ * (ldp + ldm);
    wbuf.ensure(mixed ? (pel + 1) / 2 : pel);
    wbuf2.ensure(mixed ? (wel + 1) / 2 : wel);
    scrC.ensure((size_t)nhp * chunk * np_);
    scrC2.ensure((size_t)std::max<long>(1, nhm) * chunk * np_);
    scrK.ensure(kSplitScratch);
    for (int c0 = 0; c0 < np_; c0 += (int)chunk) {
      const int c1 = std::min<int>(np_, c0 + (int)chunk);
      const int rows = c1 - c0;
      const long pairs = (long)rows * c1;
      GemmArgs g;
      g.M = rows * np_;
      g.N = c1 * np_;
      g.K = nx;
      g.lda = nx;
      g.ldb = nx;
      g.ldc = (long)c1 * np_;
      g.site = 1;
      GemmArgs hp, hm;
      hp.M = (int)nhp;
      hp.N = (int)pairs;
      hp.K = (int)ldp;
      hp.lda = ldp;
      hp.ldb = ldp;
      hp.C = scrC.p;
      hp.ldc = pairs;
      hp.site = 1;
      hm = hp;
      hm.M = (int)nhm;
      hm.K = (int)ldm;
      hm.lda = ldm;
      hm.ldb = ldm;
      hm.C = scrC2.p;
      if (!mixed) {
        g.C = wbuf2.p;
        HIPCHK(ric::gemm_nt_f64(g, BT.p + (long)c0 * np_ * nx, BT.p, stream, scrK.p, scrK.n));
        double* wp = wbuf.p;
        double* wm = wbuf.p + (size_t)pairs * ldp;
        HIPCHK(ric::pack_w(wbuf2.p, np_, rows, c1, wp, wm, ldp, ldm, stream));
        HIPCHK(ric::gemm_nt_f64(hp, tpd, wp, stream, scrK.p, scrK.n));
        if (nhm > 0) HIPCHK(ric::gemm_nt_f64(hm, tmd, wm, stream, scrK.p, scrK.n));
      } else {
        float* w2 = reinterpret_cast<float*>(wbuf2.p);
        HIPCHK(ric::gemm_nt_f32_out32(g, reinterpret_cast<const float*>(BT32.p) + (long)c0 * np_ * nx,
                                      reinterpret_cast<const float*>(BT32.p), w2, stream));
        float* wp = reinterpret_cast<float*>(wbuf.p);
        float* wm = wp + (size_t)pairs * ldp;
        HIPCHK(ric::pack_w_f32(w2, np_, rows, c1, wp, wm, ldp, ldm, stream));
        HIPCHK(ric::gemm_nt_f32(hp, tpf, wp, stream, scrK.p, scrK.n));
        if (nhm > 0) HIPCHK(ric::gemm_nt_f32(hm, tmf, wm, stream, scrK.p, scrK.n));
      }
      if (nhm == 0) HIPCHK(ric::fill(scrC2.p, 1, 0.0, stream));
      HIPCHK(ric::ladder_scatter_pm_add(scrC.p, scrC2.p, nh, np_, c0, c1, r2, stream));
    }
  }

  // -- ladder part of d<x, r>/dB -------------------------------------------------------------
  // With V[c,e,d,f] = sum_kl x[k,l,c,d] tau[k,l,e,f] (x, tau pair-symmetric, so V[c,e,d,f] =
  // V[d,f,c,e]): dB[X,c,e] += 2 sum_{d,f} V[c,e,d,f] B[X,d,f] over c, d, e, f in P.  V is built
  // for a chunk of c at a time and never stored whole.
  void laddergrad(double* dB, const double* x, const double* taus) {
    const long np_ = sz.na + sz.nv, nh = sz.nc + sz.na, nx = sz.naux, n = sz.ext(RG), nc = sz.nc;
    if (np_ == 0 || nh == 0) return;
    release_scratch();  // this step needs its own large buffers
    const long pp = np_ * np_, hh = nh * nh;
    lgx.ensure((size_t)pp * hh);
    lgt.ensure((size_t)pp * hh);
    // [k][l][c][d] -> [(c,d)][(k,l)]
    auto pair_major = [&](const double* in, double* out) {
      Iter it;
      it.nd = 4;
      const long ex[4] = {np_, np_, nh, nh}, so[4] = {np_ * hh, hh, nh, 1}, si[4] = {np_, 1, nh * pp, pp};
      it.total = pp * hh;
      for (int i = 0; i < 4; ++i) {
        it.ext[i] = ex[i];
        it.so[i] = so[i];
        it.si[i] = si[i];
      }
      HIPCHK(ric::strided_copy(it, 1.0, in, 0.0, out, stream));
    };
    pair_major(x, lgx.p);
    pair_major(taus, lgt.p);
    // rows over (d,f) padded to an even length (zero tail) so the second product loads 16 bytes
    const long ppad = (pp + 1) / 2 * 2;
    lgb.ensure((size_t)nx * ppad);
    if (ppad != pp) HIPCHK(ric::fill(lgb.p, nx * ppad, 0.0, stream));
    {  // B[X][P][P] contiguous over (d,f)
      Iter it;
      it.nd = 3;
      const long ex[3] = {nx, np_, np_}, so[3] = {ppad, np_, 1}, si[3] = {n * n, n, 1};
      it.total = nx * pp;
      for (int i = 0; i < 3; ++i) {
        it.ext[i] = ex[i];
        it.so[i] = so[i];
        it.si[i] = si[i];
      }
      HIPCHK(ric::strided_copy(it, 1.0, Bp + nc * n + nc, 0.0, lgb.p, stream));
    }
    long chunk = std::max<long>(1, (long)(1.4e9 / ((double)np_ * ppad)));
    chunk = std::min(chunk, np_);
    wbuf.ensure((size_t)chunk * np_ * ppad);
    wbuf2.ensure((size_t)chunk * np_ * pp);
    scrC.ensure((size_t)chunk * np_ * nx);
    scrK.ensure(kSplitScratch);
    if (ppad != pp) HIPCHK(ric::fill(wbuf.p, chunk * np_ * ppad, 0.0, stream));  // pad columns stay zero
    for (long c0 = 0; c0 < np_; c0 += chunk) {
      const long rows = std::min(chunk, np_ - c0);
      GemmArgs g1;  // V1[(c,d)][(e,f)]
      g1.M = (int)(rows * np_);
      g1.N = (int)pp;
      g1.K = (int)hh;
      g1.lda = hh;
      g1.ldb = hh;
      g1.C = wbuf2.p;
      g1.ldc = pp;
      HIPCHK(ric::gemm_nt_f64(g1, lgx.p + c0 * np_ * hh, lgt.p, stream, scrK.p, scrK.n));
      {  // V2[(c,e)][(d,f)] <- V1[(c,d)][(e,f)], rows of length ppad
        Iter it;
        it.nd = 4;
        const long ex[4] = {rows, np_, np_, np_}, so[4] = {np_ * ppad, ppad, np_, 1}, si[4] = {np_ * pp, np_, pp, 1};
        it.total = rows * np_ * pp;
        for (int i = 0; i < 4; ++i) {
          it.ext[i] = ex[i];
          it.so[i] = so[i];
          it.si[i] = si[i];
        }
        HIPCHK(ric::strided_copy(it, 1.0, wbuf2.p, 0.0, wbuf.p, stream));
      }
      GemmArgs g2;  // C[(c,e)][X] = 2 V2 . Bpp^T
      g2.M = (int)(rows * np_);
      g2.N = (int)nx;
      g2.K = (int)ppad;
      g2.alpha = 2.0;
      g2.lda = ppad;
      g2.ldb = ppad;
      g2.C = scrC.p;
      g2.ldc = nx;
      HIPCHK(ric::gemm_nt_f64(g2, wbuf.p, lgb.p, stream, scrK.p, scrK.n));
      {  // dB[X][nc + c][nc + e] += C[(c,e)][X]
        Iter it;
        it.nd = 3;
        const long ex[3] = {nx, rows, np_}, so[3] = {n * n, n, 1}, si[3] = {1, np_ * nx, nx};
        it.total = nx * rows * np_;
        for (int i = 0; i < 3; ++i) {
          it.ext[i] = ex[i];
          it.so[i] = so[i];
          it.si[i] = si[i];
        }
        HIPCHK(ric::strided_copy(it, 1.0, scrC.p, 1.0, dB + (nc + c0) * n + nc, stream));
      }
    }
  }

  // Give back the idle pool blocks and the work buffers (regrown on demand); only between
  // operations, after the stream has drained.
  void release_scratch() {
    HIPCHK(hipStreamSynchronize(stream));
    pool.release_idle();
    for (DevBuf* b : {&scrA, &scrB, &scrC, &scrC2, &wbuf, &wbuf2, &dfa, &dfb, &dfz, &lgx, &lgt, &lgb}) b->release();
  }

  // -- plan execution -----------------------------------------------------------------------
  // RIC_PROFILE=1: per-operation-kind device time (synchronizes after every operation)
  bool profile = getenv("RIC_PROFILE") != nullptr;
  bool profile_ops = profile && std::string(getenv("RIC_PROFILE")) == "2";  // also each operation over 20 ms
  std::map<std::string, std::pair<double, long>> prof;

  // RIC_PROGRESS=1: one stderr line when each expensive phase of a plan section ends
  bool progress = getenv("RIC_PROGRESS") != nullptr;
  std::set<const std::vector<Op>*> warmed;

  // chunked execution of a LOOP body: the intermediate's leading index runs over [s, s + len)
  // elements of one chunk of the intermediate (RIC_LOOP_BUDGET overrides, e.g. to test many chunks)
  double loop_budget = getenv("RIC_LOOP_BUDGET") ? std::atof(getenv("RIC_LOOP_BUDGET")) : 1.5e9;
  struct Loop {
    bool on = false;
    int slot = -1;
    long n = 0, s = 0, len = 0, lenmax = 0, rest = 1;
    double* buf = nullptr;
  } loop;

  // Inside a LOOP: the label that the chunked intermediate carries in its leading dimension is
  // restricted to the current chunk in every operand of the operation.
  void restrict_to_chunk(const Op& op, View* v, int nv) {
    if (!loop.on) return;
    int lab = -1;
    for (size_t k = 0; k < op.o.size(); ++k)
      if (op.o[k].slot == loop.slot) lab = op.o[k].lab.at(0);
    if (lab < 0) return;
    for (int k = 0; k < nv; ++k) {
      const int d = v[k].find(lab);
      if (d < 0) continue;
      if (v[k].ext[d] != loop.n) throw Err(RIC_E_PLAN, "chunked label does not span its full range");
      if (v[k].p) v[k].p += loop.s * v[k].str[d];
      v[k].ext[d] = loop.len;
    }
  }

  // populate the intermediate pool with every size the plan allocates (no kernels)
  void warm_pool(std::vector<Op>& ops) {
    for (Op& op : ops) {
      if (op.chunked) continue;
      if (op.kind == K_ALLOC) {
        slots[op.slot].decl = op.decl;
        slots[op.slot].ptr = pool.get((size_t)slot_elems(op.slot));
      } else if (op.kind == K_FREE) {
        pool.put(slots[op.slot].ptr, (size_t)slot_elems(op.slot));
        slots[op.slot].ptr = nullptr;
      }
    }
  }

  // Operations of a section kept under a term mask (ric_residual).  The ladder block, ALLOC TAU
  // to FREE TAU, runs as a whole or not at all.  Outside it, the operations that act on the
  // outputs alone (zeroing, symmetrizing and masking R1 and R2) always run; everything else is
  // a non-ladder term.
  bool keep_op(const std::vector<Op>& ops, size_t i, unsigned mask) const {
    if ((mask & (RIC_TERMS_LADDER | RIC_TERMS_NONLADDER)) == (RIC_TERMS_LADDER | RIC_TERMS_NONLADDER)) return true;
    auto it = ladder_block.find(&ops);
    if (it != ladder_block.end() && i >= it->second.first && i <= it->second.second)
      return (mask & RIC_TERMS_LADDER) != 0;
    const Op& op = ops[i];
    auto output = [&](int slot) { return slot >= 0 && (slots[slot].name == "R1" || slots[slot].name == "R2"); };
    if ((op.kind == K_ZERO || op.kind == K_SYMM || op.kind == K_SYMHALF) && output(op.slot)) return true;
    if (op.kind == K_MASK && output(op.slot) && output(op.slot2)) return true;
    return (mask & RIC_TERMS_NONLADDER) != 0;
  }

  // Device memory of a slot that an operation addresses directly; an operation on a tensor
  // that holds no memory (freed, or never allocated) is a plan error, not a launch.
  double* live(int slot) {
    double* p = slots.at(slot).ptr;
    if (!p && slot_elems(slot) > 0) throw Err(RIC_E_STATE, "tensor " + slots[slot].name + " is not available");
    return p;
  }

  void run(std::vector<Op>& ops, unsigned mask = RIC_TERMS_ALL) {
    if (!warmed.count(&ops)) {  // first run of this section: its intermediates enter the pool
      warm_pool(ops);
      warmed.insert(&ops);
    }
    hipEvent_t pa = nullptr, pb = nullptr;
    auto t_start = std::chrono::steady_clock::now();
    double flops_done = 0.0;
    int big_done = 0;
    if (profile) {
      HIPCHK(hipEventCreate(&pa));
      HIPCHK(hipEventCreate(&pb));
    }
    static const char* kname[] = {"ZERO", "ALLOC", "FREE", "CONTRACT", "CONTRACT0", "ADD", "DFC", "SYMM",
                                  "LADDER", "MASK", "SYMHALF", "LADDERGRAD", "LOOP", "ENDLOOP"};
    auto step = [&](Op& op) {
      if (profile) HIPCHK(hipEventRecord(pa, stream));
      switch (op.kind) {
        case K_ALLOC: {
          Slot& s = slots[op.slot];
          s.decl = op.decl;
          if (op.chunked) {
            loop.buf = pool.get((size_t)(loop.lenmax * loop.rest));
            s.ptr = loop.buf - loop.s * loop.rest;  // leading index i lives at buf + (i - s) * rest
          } else {
            s.ptr = pool.get((size_t)slot_elems(op.slot));
          }
          break;
        }
        case K_FREE: {
          Slot& s = slots[op.slot];
          if (op.chunked) pool.put(loop.buf, (size_t)(loop.lenmax * loop.rest));
          else pool.put(s.ptr, (size_t)slot_elems(op.slot));
          s.ptr = nullptr;
          break;
        }
        case K_ZERO: {
          Slot& s = slots[op.slot];
          if (accumulate_theta && (s.name == "dF" || s.name == "dB")) break;
          if (op.chunked) HIPCHK(ric::fill(loop.buf, loop.len * loop.rest, 0.0, stream));
          else HIPCHK(ric::fill(live(op.slot), slot_elems(op.slot), 0.0, stream));
          break;
        }
        case K_CONTRACT:
        case K_CONTRACT0: {
          View v[3] = {view(op.o[0]), view(op.o[1]), view(op.o[2])};
          restrict_to_chunk(op, v, 3);
          contract(v[0], op.alpha, v[1], v[2], op.kind == K_CONTRACT0, true);
          break;
        }
        case K_ADD: {
          View v[2] = {view(op.o[0]), view(op.o[1])};
          restrict_to_chunk(op, v, 2);
          axpby(v[0], op.alpha, v[1], 1.0);
          break;
        }
        case K_DFC: {
          View v[4] = {view(op.o[0]), view(op.o[1]), view(op.o[2]), view(op.o[3])};
          restrict_to_chunk(op, v, 4);
          dfc(v[0], op.alpha, v[1], v[2], v[3]);
          break;
        }
        case K_LOOP:
        case K_ENDLOOP:
          break;
        case K_SYMM:
          HIPCHK(ric::symmetrize_pairs(live(op.slot), sz.nc + sz.na, sz.na + sz.nv, stream));
          break;
        case K_SYMHALF:
          HIPCHK(ric::symmetrize_pairs_scaled(live(op.slot), sz.nc + sz.na, sz.na + sz.nv, 0.5, stream));
          break;
        case K_LADDER: {
          HIPCHK(hipEventRecord(ev[0], stream));
          ladder(live(op.slot2), live(op.slot));
          HIPCHK(hipEventRecord(ev[1], stream));
          ladder_ran = true;
          break;
        }
        case K_LADDERGRAD:
          laddergrad(live(op.slot), live(op.slot2), live(op.slot3));
          break;
        case K_MASK:
          HIPCHK(ric::mask_active(live(op.slot), live(op.slot2), sz.nc, sz.na, sz.nv, stream));
          break;
      }
      if (progress && (op.kind == K_LADDER || op.kind == K_LADDERGRAD || op.kind == K_DFC ||
                       ((op.kind == K_CONTRACT || op.kind == K_CONTRACT0) && op_flops(op) > 5e13))) {
        // report after the operation has finished on the device
        HIPCHK(hipStreamSynchronize(stream));
        ++big_done;
        const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        if (op.kind == K_LADDER || op.kind == K_LADDERGRAD || big_done % 16 == 0)
          fprintf(stderr, "  [ric] %s done: %d large operations, %.1f s\n", kind_name(op.kind), big_done, el);
      }
      if (profile) {
        HIPCHK(hipEventRecord(pb, stream));
        HIPCHK(hipEventSynchronize(pb));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, pa, pb));
        std::string key = kname[op.kind];
        if (op.kind == K_CONTRACT || op.kind == K_CONTRACT0 || op.kind == K_DFC) {
          long big = 0;
          for (auto& o : op.o) {
            long e = 1;
            for (Rng r : o.sub) e *= sz.ext(r);
            big = std::max(big, e);
          }
          key += big > 100000000L ? "/big" : big > 1000000L ? "/mid" : "/small";
        }
        auto& pr = prof[key];
        pr.first += ms;
        pr.second += 1;
        if (profile_ops && ms > 20.f)
          fprintf(stderr, "  RIC_OP %9.2f ms %9.2f TF/s  %s\n", ms, op_flops(op) / (ms * 1e-3) / 1e12,
                  op.text.empty() ? kname[op.kind] : op.text.c_str());
      }
    };
    for (size_t oi = 0; oi < ops.size(); ++oi) {
      Op& op = ops[oi];
      if (op.kind != K_LOOP) {
        if (keep_op(ops, oi, mask)) step(op);
        continue;
      }
      // the body runs once per chunk of the leading dimension of the chunked intermediate
      const size_t end = (size_t)op.slot3;
      if (!keep_op(ops, oi, mask)) {
        oi = end;
        continue;
      }
      const auto& decl = slots[op.slot].decl;
      long n = sz.ext(decl.at(0)), rest = 1;
      for (size_t d = 1; d < decl.size(); ++d) rest *= sz.ext(decl[d]);
      const long lenmax = std::min<long>(std::max<long>(n, 1), std::max<long>(1, (long)(loop_budget / std::max<long>(rest, 1))));
      for (long s0 = 0; s0 < n; s0 += lenmax) {
        loop.on = true;
        loop.slot = op.slot;
        loop.n = n;
        loop.s = s0;
        loop.len = std::min(lenmax, n - s0);
        loop.lenmax = lenmax;
        loop.rest = rest;
        for (size_t k = oi + 1; k < end; ++k) step(ops[k]);
      }
      loop.on = false;
      oi = end;
    }
    if (profile) {
      for (auto& kv : prof) fprintf(stderr, "  RIC_PROFILE %-16s %10.3f ms  %6ld ops\n", kv.first.c_str(), kv.second.first,
                                    kv.second.second);
      prof.clear();
      (void)hipEventDestroy(pa);
      (void)hipEventDestroy(pb);
    }
  }

  static const char* kind_name(Kind k) {
    static const char* n[] = {"ZERO", "ALLOC", "FREE", "CONTRACT", "CONTRACT0", "ADD", "DFC", "SYMM",
                              "LADDER", "MASK", "SYMHALF", "LADDERGRAD", "LOOP", "ENDLOOP"};
    return n[k];
  }

  double op_flops(const Op& op) const {
    std::map<int, long> ext;
    for (const auto& o : op.o)
      for (size_t i = 0; i < o.lab.size(); ++i) ext[o.lab[i]] = sz.ext(o.sub[i]);
    double f = 2.0;
    for (auto& kv : ext) f *= (double)kv.second;
    return f;
  }

  void bind(const char* name, const double* p) { slots[slot_of.at(name)].ptr = const_cast<double*>(p); }

  void require_loaded() {
    if (!spaces) throw Err(RIC_E_STATE, "ric_set_spaces has not been called");
    if (!have_f || !have_B) throw Err(RIC_E_STATE, "Fock matrix and DF factors must be loaded");
    if (sz.na > 0 && !have_rdm) throw Err(RIC_E_STATE, "RDMs must be loaded when na > 0");
  }
};

namespace {

std::string default_plan_path() {
  Dl_info info;
  if (dladdr(reinterpret_cast<void*>(&default_plan_path), &info) && info.dli_fname) {
    std::string p(info.dli_fname);
    auto k = p.rfind('/');
    std::string dir = k == std::string::npos ? "." : p.substr(0, k);
    return dir + "/plan.txt";
  }
  return "plan.txt";
}

}  // namespace

namespace {
int guard(ric_ctx* ctx, const std::function<void()>& fn) {
  if (!ctx) return RIC_E_ARG;
  try {
    HIPCHK(hipSetDevice(ctx->device));
    (void)hipGetLastError();  // clear a stale error left by an earlier failed call
    fn();
    ctx->err.clear();
    return RIC_OK;
  } catch (const Err& e) {
    ctx->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return RIC_E_ARG;
  }
}
}  // namespace

extern "C" {

int ric_create(ric_ctx** out, int device, void* hip_stream, const char* plan_path) {
  if (!out) return RIC_E_ARG;
  *out = nullptr;
  auto* ctx = new (std::nothrow) ric_ctx();
  if (!ctx) return RIC_E_OOM;
  ctx->device = device;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  int rc = guard(ctx, [&] {
    for (auto& e : ctx->ev) HIPCHK(hipEventCreate(&e));
    ctx->noalloc = noalloc_scratch(device);   // guard() made `device` current
    ctx->load_plan(plan_path ? std::string(plan_path) : default_plan_path());
  });
  if (rc != RIC_OK) {
    fprintf(stderr, "ric_create: %s\n", ctx->err.c_str());
    delete ctx;
    return rc;
  }
  *out = ctx;
  return RIC_OK;
}

void ric_destroy(ric_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
}

int ric_set_spaces(ric_ctx* ctx, int nc, int na, int nv, int naux) {
  return guard(ctx, [&] {
    if (nc < 0 || na < 0 || nv < 0 || naux < 1 || na > 16 || nc + na < 1 || na + nv < 1)
      throw Err(RIC_E_ARG, "invalid orbital space sizes");
    ctx->sz = Sizes{nc, na, nv, naux};
    ctx->Bp = nullptr;
    ctx->drop_shadows();
    ctx->spaces = true;
    ctx->have_f = ctx->have_B = ctx->have_rdm = false;
  });
}

int ric_load_fock(ric_ctx* ctx, const double* f) {
  return guard(ctx, [&] {
    if (!ctx->spaces) throw Err(RIC_E_STATE, "ric_set_spaces has not been called");
    if (!f) throw Err(RIC_E_ARG, "null Fock matrix");
    const long n = ctx->sz.ext(RG);
    ctx->f.ensure(n * n);
    HIPCHK(hipMemcpyAsync(ctx->f.p, f, n * n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    ctx->eps.ensure(n);
    HIPCHK(ric::fock_diagonal(ctx->f.p, (int)n, ctx->eps.p, ctx->stream));
    ctx->bind("f", ctx->f.p);
    ctx->have_f = true;
  });
}

int ric_load_df(ric_ctx* ctx, const double* B, int borrow) {
  return guard(ctx, [&] {
    if (!ctx->spaces) throw Err(RIC_E_STATE, "ric_set_spaces has not been called");
    if (!B) throw Err(RIC_E_ARG, "null DF factors");
    const Sizes& s = ctx->sz;
    const long n = s.ext(RG), nx = s.naux, nc = s.nc, np_ = s.ext(RP);
    ctx->drop_shadows();
    if (borrow) {
      ctx->B.release();   // the caller's array is used in place and must outlive its use here
      ctx->Bp = B;
    } else {
      ctx->B.ensure((size_t)nx * n * n);
      HIPCHK(hipMemcpyAsync(ctx->B.p, B, (size_t)nx * n * n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
      ctx->Bp = ctx->B.p;
    }
    ctx->bind("B", ctx->Bp);
    // ladder operand BT[c][e][X] = B[X][nc + c][nc + e]
    ctx->BT.ensure((size_t)np_ * np_ * nx);
    {
      View v;
      v.p = const_cast<double*>(ctx->Bp) + nc * n + nc;
      v.nd = 3;
      v.ext[0] = nx; v.str[0] = n * n; v.lab[0] = 0;
      v.ext[1] = np_; v.str[1] = n; v.lab[1] = 1;
      v.ext[2] = np_; v.str[2] = 1; v.lab[2] = 2;
      ctx->gather(v, {1, 2, 0}, ctx->BT.p, nullptr);
      ctx->BT32.ensure(((size_t)np_ * np_ * nx + 1) / 2);
      ctx->gather(v, {1, 2, 0}, nullptr, reinterpret_cast<float*>(ctx->BT32.p));
    }
    // stored integral blocks (pr|qs) with at most two particle indices
    std::map<std::string, int> lab;
    auto mk = [&](const char* nm, const char* decl, DevBuf& buf) {
      std::vector<Rng> d;
      for (const char* c = decl; *c; ++c) d.push_back(rng_of(*c));
      long e = 1;
      for (Rng r : d) e *= s.ext(r);
      buf.ensure((size_t)e);
      ctx->bind(nm, buf.p);
      // (pr|qs) = sum_X B[X,p,r] B[X,q,s]
      Opd o, b1, b2;
      o.slot = ctx->slot_of.at(nm);
      o.sub = d;
      o.lab = {1, 2, 3, 4};
      b1.slot = ctx->slot_of.at("B");
      b1.sub = {RX, d[0], d[1]};
      b1.lab = {0, 1, 2};
      b2.slot = ctx->slot_of.at("B");
      b2.sub = {RX, d[2], d[3]};
      b2.lab = {0, 3, 4};
      ctx->contract(ctx->view(o), 1.0, ctx->view(b1), ctx->view(b2), true, false);
    };
    mk("I4", "HHHH", ctx->I4);
    mk("I3", "HHHP", ctx->I3);
    mk("IJ", "HHPP", ctx->IJ);
    mk("IK", "HPHP", ctx->IK);
    ctx->have_B = true;
  });
}

int ric_load_rdms(ric_ctx* ctx, const double* G1, const double* G2, const double* G3) {
  return guard(ctx, [&] {
    if (!ctx->spaces) throw Err(RIC_E_STATE, "ric_set_spaces has not been called");
    const long na = ctx->sz.na;
    if (na == 0) {
      ctx->have_rdm = true;
      return;
    }
    if (!G1 || !G2 || !G3) throw Err(RIC_E_ARG, "null RDM");
    const long n2 = na * na, n4 = n2 * n2, n6 = n4 * n2;
    ctx->g1.ensure(n2);
    ctx->g2.ensure(n4);
    ctx->g3.ensure(n6);
    HIPCHK(hipMemcpyAsync(ctx->g1.p, G1, n2 * 8, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->g2.p, G2, n4 * 8, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->g3.p, G3, n6 * 8, hipMemcpyDeviceToDevice, ctx->stream));
    ctx->ga.ensure(n2);
    ctx->ea.ensure(n2);
    ctx->l2.ensure(n4);
    ctx->k2.ensure(n4);
    ctx->l3.ensure(n6);
    ctx->k3.ensure(n6);
    HIPCHK(ric::prepare_cumulants(ctx->g1.p, ctx->g2.p, ctx->g3.p, (int)na, ctx->ga.p, ctx->ea.p, ctx->l2.p,
                                  ctx->k2.p, ctx->l3.p, ctx->k3.p, ctx->stream));
    ctx->bind("gA", ctx->ga.p);
    ctx->bind("eA", ctx->ea.p);
    ctx->bind("K2", ctx->k2.p);
    ctx->bind("K3", ctx->k3.p);
    ctx->have_rdm = true;
  });
}

int ric_residual(ric_ctx* ctx, const double* T1, const double* T2, double* R1, double* R2, int precision,
                 unsigned term_mask) {
  return guard(ctx, [&] {
    ctx->require_loaded();
    if (!T1 || !T2 || !R1 || !R2) throw Err(RIC_E_ARG, "null amplitude/residual pointer");
    if (precision != RIC_FP64 && precision != RIC_FP32MIX) throw Err(RIC_E_ARG, "bad precision");
    if (term_mask & ~(unsigned)RIC_TERMS_ALL) throw Err(RIC_E_ARG, "unknown term group bits");
    const bool lin = term_mask & RIC_TERMS_LINEAR, quad = term_mask & RIC_TERMS_QUADRATIC;
    if (!(lin || quad) || !(term_mask & (RIC_TERMS_LADDER | RIC_TERMS_NONLADDER)))
      throw Err(RIC_E_ARG, "term mask selects no terms");
    const char* sec = lin && quad ? "residual" : lin ? "residual_lin" : "residual_quad";
    ctx->precision = precision;
    ctx->use_ladder_budget(ric_ctx::kLadderBudgetForward);
    ctx->bind("T1", T1);
    ctx->bind("T2", T2);
    ctx->bind("R1", R1);
    ctx->bind("R2", R2);
    ctx->ladder_ran = false;
    HIPCHK(hipEventRecord(ctx->ev[2], ctx->stream));
    if (precision == RIC_FP32MIX) {
      // FP32 copies of the operands large products read in place: the amplitudes at every call
      // (inside the timed region), the stored blocks once per load; made after the section's
      // intermediates hold their memory, and only where the device has room
      auto& ops = ctx->sections.at(sec);
      if (!ctx->warmed.count(&ops)) {
        ctx->warm_pool(ops);
        ctx->warmed.insert(&ops);
      }
      ctx->make_shadow("T2", ctx->sh_t2);
      ctx->make_shadow("T1", ctx->sh_t1);
      ctx->static_shadows();
    }
    ctx->run(ctx->sections.at(sec), term_mask);
    ctx->slots[ctx->slot_of.at("T1")].ptr32 = nullptr;
    ctx->slots[ctx->slot_of.at("T2")].ptr32 = nullptr;
    HIPCHK(hipEventRecord(ctx->ev[3], ctx->stream));
    HIPCHK(hipEventSynchronize(ctx->ev[3]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]));
    ctx->total_ms = ms;
    ms = 0.f;
    if (ctx->ladder_ran) HIPCHK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
    ctx->ladder_ms = ms;
  });
}

int ric_update(ric_ctx* ctx, double* T1, double* T2, const double* R1, const double* R2, double s,
               double* step_norm2) {
  return guard(ctx, [&] {
    ctx->require_loaded();
    if (!T1 || !T2 || !R1 || !R2) throw Err(RIC_E_ARG, "null amplitude/residual pointer");
    if (!(s >= 0.0)) throw Err(RIC_E_ARG, "flow parameter must be >= 0");
    ctx->red.ensure(ric::kReducePartials);
    ctx->Edev.ensure(4);
    HIPCHK(ric::ric_update_kernel(T1, T2, R1, R2, ctx->eps.p, ctx->sz.nc, ctx->sz.na, ctx->sz.nv, s, ctx->red.p,
                                  ctx->Edev.p + 1, ctx->stream));
    double v = 0.0;
    HIPCHK(hipMemcpyAsync(&v, ctx->Edev.p + 1, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (!std::isfinite(v)) throw Err(RIC_E_NONFINITE, "non-finite amplitude step");
    if (step_norm2) *step_norm2 = v;
  });
}

int ric_update_noalloc(ric_ctx* ctx, double* T1, double* T2, const double* R1, const double* R2, double s,
                       double* step_norm2) {
  return guard(ctx, [&] {
    ctx->require_loaded();
    if (!T1 || !T2 || !R1 || !R2) throw Err(RIC_E_ARG, "null amplitude/residual pointer");
    if (!(s >= 0.0)) throw Err(RIC_E_ARG, "flow parameter must be >= 0");
    // the same kernels as ric_update, with the reduction's partial sums and result in `scratch`
    constexpr size_t need = (size_t)ric::kReducePartials + 1;
    static_assert(need <= kNoAllocDoubles, "reduction partials exceed the allocation-free scratch");
    if (need > kNoAllocDoubles) throw Err(RIC_E_ARG, "reduction needs more than the allocation-free scratch holds");
    if (!ctx->noalloc) throw Err(RIC_E_STATE, "allocation-free scratch not set up");
    double* partial = ctx->noalloc;
    double* result = ctx->noalloc + ric::kReducePartials;
    HIPCHK(ric::ric_update_kernel(T1, T2, R1, R2, ctx->eps.p, ctx->sz.nc, ctx->sz.na, ctx->sz.nv, s, partial, result,
                                  ctx->stream));
    double v = 0.0;
    HIPCHK(hipMemcpyAsync(&v, result, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (!std::isfinite(v)) throw Err(RIC_E_NONFINITE, "non-finite amplitude step");
    if (step_norm2) *step_norm2 = v;
  });
}

int ric_energy(ric_ctx* ctx, const double* T1, const double* T2, double* e_corr, double* e0) {
  return guard(ctx, [&] {
    ctx->require_loaded();
    if (!T1 || !T2 || !e_corr) throw Err(RIC_E_ARG, "null pointer");
    ctx->bind("T1", T1);
    ctx->bind("T2", T2);
    ctx->Edev.ensure(4);
    ctx->bind("E", ctx->Edev.p);
    ctx->precision = RIC_FP64;
    ctx->drop_shadows();   // FP64 only: return the mixed path's FP32 operand copies
    HIPCHK(ric::fill(ctx->Edev.p, 1, 0.0, ctx->stream));
    ctx->run(ctx->sections.at("energy"));
    if (e0) {
      const double* g1 = ctx->sz.na ? ctx->g1.p : nullptr;
      const double* g2 = ctx->sz.na ? ctx->g2.p : nullptr;
      HIPCHK(ric::reference_energy(ctx->f.p, (int)ctx->sz.ext(RG), ctx->I4.p, ctx->sz.nc, ctx->sz.na, g1, g2,
                                   ctx->Edev.p + 2, ctx->stream));
    }
    double h[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(h, ctx->Edev.p, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (!std::isfinite(h[0])) throw Err(RIC_E_NONFINITE, "non-finite energy");
    *e_corr = h[0];
    if (e0) *e0 = h[2];
  });
}

int ric_ladder(ric_ctx* ctx, const double* tau, double* R2, int precision) {
  return guard(ctx, [&] {
    if (!ctx->spaces || !ctx->have_B) throw Err(RIC_E_STATE, "DF factors must be loaded");
    if (!tau || !R2) throw Err(RIC_E_ARG, "null pointer");
    if (precision != RIC_FP64 && precision != RIC_FP32MIX) throw Err(RIC_E_ARG, "bad precision");
    ctx->precision = precision;
    ctx->use_ladder_budget(ric_ctx::kLadderBudgetForward);
    HIPCHK(hipEventRecord(ctx->ev[0], ctx->stream));
    ctx->ladder(tau, R2);
    HIPCHK(hipEventRecord(ctx->ev[1], ctx->stream));
    HIPCHK(hipEventSynchronize(ctx->ev[1]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
    ctx->ladder_ms = ms;
    ctx->total_ms = ms;
  });
}

int ric_adjoint_residual(ric_ctx* ctx, const double* T1, const double* T2, const double* X1, const double* X2,
                         double* dT1, double* dT2, double* dF, double* dB, int accumulate) {
  return guard(ctx, [&] {
    ctx->require_loaded();
    if (!T1 || !T2 || !X1 || !X2 || !dT1 || !dT2) throw Err(RIC_E_ARG, "null amplitude/cotangent pointer");
    if ((dF == nullptr) != (dB == nullptr)) throw Err(RIC_E_ARG, "dF and dB must both be given or both be NULL");
    const long nh = ctx->sz.nc + ctx->sz.na, np_ = ctx->sz.na + ctx->sz.nv;
    const long n1 = nh * np_, n2 = n1 * n1;
    ctx->precision = RIC_FP64;
    ctx->use_ladder_budget(ric_ctx::kLadderBudgetAdjoint);
    ctx->drop_shadows();   // the FP32 operand copies of the mixed path are not needed here
    // cotangents of the masked residuals: R1 as given, R2 through its pair-symmetric part
    ctx->xr1.ensure(n1);
    ctx->xl.ensure(n2);
    HIPCHK(hipMemcpyAsync(ctx->xr1.p, X1, n1 * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->xl.p, X2, n2 * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ric::symmetrize_pairs_scaled(ctx->xl.p, (int)nh, (int)np_, 0.5, ctx->stream));
    HIPCHK(ric::mask_active(ctx->xr1.p, ctx->xl.p, ctx->sz.nc, ctx->sz.na, ctx->sz.nv, ctx->stream));
    ctx->bind("T1", T1);
    ctx->bind("T2", T2);
    ctx->bind("XR1", ctx->xr1.p);
    ctx->bind("XL", ctx->xl.p);
    ctx->bind("dT1", dT1);
    ctx->bind("dT2", dT2);
    ctx->run(ctx->sections.at("adjoint_t"));
    if (dF) {
      ctx->bind("dF", dF);
      ctx->bind("dB", dB);
      ctx->release_scratch();  // the (f, B) part holds its own, larger intermediates
      ctx->accumulate_theta = accumulate != 0;
      try {
        ctx->run(ctx->sections.at("adjoint_theta"));
      } catch (...) {
        ctx->accumulate_theta = false;
        throw;
      }
      ctx->accumulate_theta = false;
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

int ric_energy_gradient(ric_ctx* ctx, const double* T1, const double* T2, double* dT1, double* dT2, double* dF,
                        double* dB) {
  return guard(ctx, [&] {
    ctx->require_loaded();
    if (!T1 || !T2 || !dT1 || !dT2 || !dF || !dB) throw Err(RIC_E_ARG, "null pointer");
    ctx->precision = RIC_FP64;
    ctx->use_ladder_budget(ric_ctx::kLadderBudgetAdjoint);
    ctx->drop_shadows();   // the FP32 operand copies of the mixed path are not needed here
    ctx->bind("T1", T1);
    ctx->bind("T2", T2);
    ctx->bind("dT1", dT1);
    ctx->bind("dT2", dT2);
    ctx->bind("dF", dF);
    ctx->bind("dB", dB);
    ctx->run(ctx->sections.at("energy_grad"));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

int ric_lambda_update(ric_ctx* ctx, double* L1, double* L2, const double* G1, const double* G2, const double* J1,
                      const double* J2, double s, double* step_norm2) {
  return guard(ctx, [&] {
    ctx->require_loaded();
    if (!L1 || !L2 || !G1 || !G2 || !J1 || !J2) throw Err(RIC_E_ARG, "null pointer");
    if (!(s >= 0.0)) throw Err(RIC_E_ARG, "flow parameter must be >= 0");
    ctx->red.ensure(ric::kReducePartials);
    ctx->Edev.ensure(4);
    HIPCHK(ric::lambda_update(L1, L2, G1, G2, J1, J2, ctx->eps.p, ctx->sz.nc, ctx->sz.na, ctx->sz.nv, s, ctx->red.p,
                              ctx->Edev.p + 3, ctx->stream));
    double v = 0.0;
    HIPCHK(hipMemcpyAsync(&v, ctx->Edev.p + 3, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (!std::isfinite(v)) throw Err(RIC_E_NONFINITE, "non-finite Lagrangian step");
    if (step_norm2) *step_norm2 = v;
  });
}

int ric_flow_scale(ric_ctx* ctx, const double* L1, const double* L2, double s, double* O1, double* O2) {
  return guard(ctx, [&] {
    ctx->require_loaded();
    if (!L1 || !L2 || !O1 || !O2) throw Err(RIC_E_ARG, "null pointer");
    if (!(s >= 0.0)) throw Err(RIC_E_ARG, "flow parameter must be >= 0");
    HIPCHK(ric::flow_scale(L1, L2, ctx->eps.p, ctx->sz.nc, ctx->sz.na, ctx->sz.nv, s, O1, O2, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

int ric_flow_fock_gradient(ric_ctx* ctx, const double* T1, const double* T2, const double* R1, const double* R2,
                           const double* L1, const double* L2, double s, double* dF) {
  return guard(ctx, [&] {
    ctx->require_loaded();
    if (!T1 || !T2 || !R1 || !R2 || !L1 || !L2 || !dF) throw Err(RIC_E_ARG, "null pointer");
    if (!(s >= 0.0)) throw Err(RIC_E_ARG, "flow parameter must be >= 0");
    HIPCHK(ric::flow_fock_gradient(T1, T2, R1, R2, L1, L2, ctx->eps.p, ctx->sz.nc, ctx->sz.na, ctx->sz.nv, s, dF,
                                   ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

int ric_build_fock(ric_ctx* ctx, const double* h, double* f) {
  return guard(ctx, [&] {
    if (!ctx->spaces || !ctx->have_B) throw Err(RIC_E_STATE, "DF factors must be loaded");
    if (ctx->sz.na > 0 && !ctx->have_rdm) throw Err(RIC_E_STATE, "RDMs must be loaded when na > 0");
    if (!h || !f) throw Err(RIC_E_ARG, "null pointer");
    const int n = (int)ctx->sz.ext(RG), nc = ctx->sz.nc, na = ctx->sz.na, nx = ctx->sz.naux;
    const long n2 = (long)n * n;
    hipStream_t st = ctx->stream;
    // f = h + sum_X B[X] (B[X] . D) - sum_i B_pi B_iq - 1/2 sum_tu Gamma_tu B_pu B_tq
    HIPCHK(hipMemcpyAsync(f, h, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    ctx->scrA.ensure((size_t)n2);
    ctx->scrB.ensure((size_t)nx);
    HIPCHK(ric::fock_weights(ctx->scrA.p, n, nc, na, na ? ctx->g1.p : nullptr, st));
    GemmArgs gd;  // d[X] = sum_pq B[X,p,q] D[p,q]
    gd.M = nx;
    gd.N = 1;
    gd.K = (int)n2;
    gd.lda = n2;
    gd.ldb = n2;
    gd.C = ctx->scrB.p;
    gd.ldc = 1;
    ctx->scrK.ensure(kSplitScratch);
    HIPCHK(ric::gemm_nt_f64(gd, ctx->Bp, ctx->scrA.p, st, ctx->scrK.p, ctx->scrK.n));
    HIPCHK(ric::column_dot(ctx->Bp, ctx->scrB.p, nx, n2, 1.0, f, st));
    // exchange with the core and active orbitals: Y[p][(X,k)] = B[X,p,k] over k in C + A, with
    // the active columns contracted with Gamma1 / 2, then f -= Y Z^T (Z the same gather unweighted)
    const int m = nc + na;
    if (m > 0) {
      ctx->scrC.ensure((size_t)n * nx * m);
      ctx->scrC2.ensure((size_t)n * nx * m);
      Iter it;  // scrC[p][X][k] = B[X][p][k]
      it.nd = 3;
      const long ex[3] = {n, nx, m}, so[3] = {(long)nx * m, m, 1}, si[3] = {n, n2, 1};
      it.total = (long)n * nx * m;
      for (int i = 0; i < 3; ++i) {
        it.ext[i] = ex[i];
        it.so[i] = so[i];
        it.si[i] = si[i];
      }
      HIPCHK(ric::strided_copy(it, 1.0, ctx->Bp, 0.0, ctx->scrC.p, st));
      // weighted copy: core columns as is, active columns Gamma1/2-contracted
      HIPCHK(hipMemcpyAsync(ctx->scrC2.p, ctx->scrC.p, (size_t)n * nx * m * sizeof(double), hipMemcpyDeviceToDevice,
                            st));
      if (na > 0) {
        GemmArgs ga;  // W[(p,X)][t] = 1/2 sum_u B[X,p,u] Gamma1[t,u]
        ga.M = n * nx;
        ga.N = na;
        ga.K = na;
        ga.alpha = 0.5;
        ga.lda = m;
        ga.ldb = na;
        ga.C = ctx->scrC2.p + nc;
        ga.ldc = m;
        HIPCHK(ric::gemm_nt_f64(ga, ctx->scrC.p + nc, ctx->g1.p, st, ctx->scrK.p, ctx->scrK.n));
      }
      GemmArgs gk;  // f[p][q] -= sum_(X,k) Y[p][(X,k)] Z[q][(X,k)]
      gk.M = n;
      gk.N = n;
      gk.K = nx * m;
      gk.alpha = -1.0;
      gk.beta = 1.0;
      gk.lda = (long)nx * m;
      gk.ldb = (long)nx * m;
      gk.C = f;
      gk.ldc = n;
      HIPCHK(ric::gemm_nt_f64(gk, ctx->scrC2.p, ctx->scrC.p, st, ctx->scrK.p, ctx->scrK.n));
    }
    HIPCHK(hipStreamSynchronize(st));
  });
}

namespace {
void copy2d(long rows, long cols, const double* in, long si0, long si1, double* out, long so0, long so1,
            hipStream_t st) {
  Iter it;
  it.nd = 2;
  it.ext[0] = rows;
  it.ext[1] = cols;
  it.si[0] = si0;
  it.si[1] = si1;
  it.so[0] = so0;
  it.so[1] = so1;
  it.total = rows * cols;
  HIPCHK(ric::strided_copy(it, 1.0, in, 0.0, out, st));
}

// x[i_1..i_k] <- sum U[j_1][i_1] .. U[j_k][i_k] x[j_1..j_k] for an m^k tensor (ut = U^T, m x m):
// k rounds of (contract the last index, then rotate it to the front)
void rotate_all_indices(double* x, double* tmp, int m, int k, const double* ut, hipStream_t st, double* scr,
                        size_t nscr) {
  long rest = 1;
  for (int i = 1; i < k; ++i) rest *= m;
  for (int r = 0; r < k; ++r) {
    GemmArgs g;
    g.M = (int)rest;
    g.N = m;
    g.K = m;
    g.lda = m;
    g.ldb = m;
    g.C = tmp;
    g.ldc = m;
    HIPCHK(ric::gemm_nt_f64(g, x, ut, st, scr, nscr));
    copy2d(m, rest, tmp, 1, m, x, rest, 1, st);  // x[t'][rest] = tmp[rest][t']
  }
}
}  // namespace

int ric_semicanonicalize(ric_ctx* ctx, double* U, double* f_out) {
  int rc = guard(ctx, [&] {
    ctx->require_loaded();
    if (!U) throw Err(RIC_E_ARG, "null U");
    const int nc = ctx->sz.nc, na = ctx->sz.na, nv = ctx->sz.nv, nx = ctx->sz.naux;
    const int n = nc + na + nv;
    const long n2 = (long)n * n;
    hipStream_t st = ctx->stream;
    if (!ctx->solver) {
      if (rocblas_create_handle(&ctx->solver) != rocblas_status_success) throw Err(RIC_E_HIP, "rocblas handle");
    }
    if (rocblas_set_stream(ctx->solver, st) != rocblas_status_success) throw Err(RIC_E_HIP, "rocblas stream");
    ctx->release_scratch();
    ctx->scrK.ensure(kSplitScratch);
    double* scr = ctx->scrK.p;
    const size_t nscr = ctx->scrK.n;
    // U: eigenvectors of the core, active and virtual diagonal blocks of f
    HIPCHK(ric::fill(U, n2, 0.0, st));
    const int mmax = std::max(nc, std::max(na, nv));
    ctx->scrA.ensure((size_t)mmax * mmax + 2 * mmax + 1);
    double* blk = ctx->scrA.p;
    double* ev = blk + (size_t)mmax * mmax;
    double* off = ev + mmax;
    rocblas_int* info = nullptr;
    HIPCHK(hipMalloc(&info, sizeof(rocblas_int)));
    const int o3[3] = {0, nc, nc + na}, m3[3] = {nc, na, nv};
    for (int b = 0; b < 3; ++b) {
      const int o = o3[b], m = m3[b];
      if (m == 0) continue;
      copy2d(m, m, ctx->f.p + (long)o * n + o, n, 1, blk, m, 1, st);
      if (rocsolver_dsyevd(ctx->solver, rocblas_evect_original, rocblas_fill_upper, m, blk, m, ev, off, info) !=
          rocblas_status_success)
        throw Err(RIC_E_HIP, "rocsolver_dsyevd");
      rocblas_int hinfo = 0;
      HIPCHK(hipMemcpyAsync(&hinfo, info, sizeof(rocblas_int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (hinfo != 0) throw Err(RIC_E_HIP, "eigensolver did not converge");
      // column-major eigenvectors: U[o + i][o + j] = blk[j * m + i], each with its entry of
      // largest magnitude positive
      copy2d(m, m, blk, 1, m, U + (long)o * n + o, n, 1, st);
      HIPCHK(ric::column_signs(U + (long)o * n + o, m, n, st));
    }
    (void)hipFree(info);
    ctx->scrB.ensure((size_t)n2 * 3);
    double* Ut = ctx->scrB.p;
    double* f1 = Ut + n2;
    double* f1t = f1 + n2;
    copy2d(n, n, U, 1, n, Ut, n, 1, st);
    GemmArgs g;  // f1 = f U
    g.M = n;
    g.N = n;
    g.K = n;
    g.lda = n;
    g.ldb = n;
    g.ldc = n;
    g.C = f1;
    HIPCHK(ric::gemm_nt_f64(g, ctx->f.p, Ut, st, scr, nscr));
    copy2d(n, n, f1, 1, n, f1t, n, 1, st);
    ctx->scrC.ensure((size_t)n2);
    g.C = ctx->scrC.p;  // f' = U^T f U
    HIPCHK(ric::gemm_nt_f64(g, Ut, f1t, st, scr, nscr));
    if (f_out) HIPCHK(hipMemcpyAsync(f_out, ctx->scrC.p, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    // B'[X] = U^T B[X] U
    ctx->wbuf.ensure((size_t)nx * n2);
    ctx->wbuf2.ensure((size_t)nx * n2);
    GemmArgs gb;  // B1[(X,p)][q'] = sum_q B[X,p,q] U[q,q']
    gb.M = nx * n;
    gb.N = n;
    gb.K = n;
    gb.lda = n;
    gb.ldb = n;
    gb.ldc = n;
    gb.C = ctx->wbuf.p;
    HIPCHK(ric::gemm_nt_f64(gb, ctx->Bp, Ut, st, scr, nscr));
    {  // B1t[X][q'][p] = B1[X][p][q']
      Iter it;
      it.nd = 3;
      const long ex[3] = {nx, n, n}, so[3] = {n2, n, 1}, si[3] = {n2, 1, n};
      it.total = (long)nx * n2;
      for (int i = 0; i < 3; ++i) {
        it.ext[i] = ex[i];
        it.so[i] = so[i];
        it.si[i] = si[i];
      }
      HIPCHK(ric::strided_copy(it, 1.0, ctx->wbuf.p, 0.0, ctx->wbuf2.p, st));
    }
    gb.C = ctx->wbuf.p;  // B'[X][q'][p'] = sum_p B1t[X][q'][p] U[p][p']
    HIPCHK(ric::gemm_nt_f64(gb, ctx->wbuf2.p, Ut, st, scr, nscr));
    // RDMs: every index rotated by the active block of U
    double* ga1 = nullptr;
    double* ga2 = nullptr;
    double* ga3 = nullptr;
    if (na > 0) {
      const long a2 = (long)na * na, a4 = a2 * a2, a6 = a4 * a2;
      ctx->dfa.ensure((size_t)(a2 + a4 + a6 + a2));
      ctx->dfb.ensure((size_t)a6);
      ga1 = ctx->dfa.p;
      ga2 = ga1 + a2;
      ga3 = ga2 + a4;
      double* uat = ga3 + a6;
      copy2d(na, na, Ut + (long)nc * n + nc, n, 1, uat, na, 1, st);
      HIPCHK(hipMemcpyAsync(ga1, ctx->g1.p, a2 * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(ga2, ctx->g2.p, a4 * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(ga3, ctx->g3.p, a6 * 8, hipMemcpyDeviceToDevice, st));
      rotate_all_indices(ga1, ctx->dfb.p, na, 2, uat, st, scr, nscr);
      rotate_all_indices(ga2, ctx->dfb.p, na, 4, uat, st, scr, nscr);
      rotate_all_indices(ga3, ctx->dfb.p, na, 6, uat, st, scr, nscr);
    }
    HIPCHK(hipStreamSynchronize(st));
    // load the rotated quantities (the copies go to the context's own buffers)
    ctx->f.ensure(n2);
    HIPCHK(hipMemcpyAsync(ctx->f.p, ctx->scrC.p, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(ric::fock_diagonal(ctx->f.p, n, ctx->eps.p, st));
    HIPCHK(hipStreamSynchronize(st));
    ctx->sc_B = ctx->wbuf.p;
    ctx->sc_g = {ga1, ga2, ga3};
  });
  if (rc != RIC_OK) return rc;
  // outside the guard: the public loaders take the rotated copies
  rc = ric_load_df(ctx, ctx->sc_B, 0);   // copied: the rotated factors sit in a work buffer
  if (rc == RIC_OK && ctx->sz.na > 0) rc = ric_load_rdms(ctx, ctx->sc_g[0], ctx->sc_g[1], ctx->sc_g[2]);
  ctx->sc_B = nullptr;
  return guard(ctx, [&] {
    if (rc != RIC_OK) throw Err(rc, ctx->err);
    ctx->release_scratch();
  });
}

int ric_vec_dot(ric_ctx* ctx, const double* a, const double* b, long n, double* out) {
  return guard(ctx, [&] {
    if (!a || !b || !out || n < 0) throw Err(RIC_E_ARG, "bad vector arguments");
    ctx->red.ensure(ric::kReducePartials);
    ctx->Edev.ensure(4);
    HIPCHK(ric::fill(ctx->Edev.p, 1, 0.0, ctx->stream));
    HIPCHK(ric::dot_accumulate(a, b, n, 1.0, ctx->Edev.p, ctx->red.p, ctx->stream));
    double v = 0.0;
    HIPCHK(hipMemcpyAsync(&v, ctx->Edev.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *out = v;
  });
}

int ric_vec_axpby(ric_ctx* ctx, double alpha, const double* x, double beta, double* y, long n) {
  return guard(ctx, [&] {
    if (!x || !y || n < 0) throw Err(RIC_E_ARG, "bad vector arguments");
    Iter it;
    it.nd = 1;
    it.ext[0] = n;
    it.so[0] = 1;
    it.si[0] = 1;
    it.total = n;
    HIPCHK(ric::strided_copy(it, alpha, x, beta, y, ctx->stream));
  });
}

int ric_layout(const ric_ctx* ctx, ric_layout_t* out) {
  if (!ctx || !out) return RIC_E_ARG;
  if (!ctx->spaces) return RIC_E_STATE;
  const Sizes& z = ctx->sz;
  const int nc = z.nc, na = z.na, nv = z.nv, nh = nc + na, np = na + nv;
  std::memset(out, 0, sizeof(*out));
  out->nc = nc;
  out->na = na;
  out->nv = nv;
  out->naux = z.naux;
  out->nh = nh;
  out->np = np;
  out->t1_elems = (long)nh * np;
  out->t2_elems = (long)nh * nh * np * np;
  // hole ranges: core [0, nc), active [nc, nh); particle ranges: active [0, na), virtual [na, np)
  struct R { int s, e; };
  const R Ch{0, nc}, Ah{nc, na}, Ap{0, na}, Vp{na, nv};
  struct Cls { const char* name; int rank; R r[4]; };
  const Cls cls[12] = {
      {"IA", 1, {Ch, Vp}},           {"IT", 1, {Ch, Ap}},           {"TA", 1, {Ah, Vp}},
      {"IJAB", 2, {Ch, Ch, Vp, Vp}}, {"IJTU", 2, {Ch, Ch, Ap, Ap}}, {"TUAB", 2, {Ah, Ah, Vp, Vp}},
      {"ITAB", 2, {Ch, Ah, Vp, Vp}}, {"ITUV", 2, {Ch, Ah, Ap, Ap}}, {"IJTA", 2, {Ch, Ch, Ap, Vp}},
      {"TUVA", 2, {Ah, Ah, Ap, Vp}}, {"ITUA1", 2, {Ch, Ah, Ap, Vp}}, {"ITUA2", 2, {Ch, Ah, Vp, Ap}}};
  out->nblocks = 12;
  for (int b = 0; b < 12; ++b) {
    ric_block_t& o = out->block[b];
    std::snprintf(o.name, sizeof(o.name), "%s", cls[b].name);
    o.rank = cls[b].rank;
    for (int i = 0; i < 2 * cls[b].rank; ++i) {
      o.start[i] = cls[b].r[i].s;
      o.extent[i] = cls[b].r[i].e;
    }
  }
  return RIC_OK;
}

int ric_diis_coefficients(const double* G, int m, double* c) {
  if (!G || !c || m < 1 || m > 32) return RIC_E_ARG;
  // bordered system [G 1; 1^T 0] [c; mu] = [0; 1], G scaled by its largest diagonal element;
  // Gaussian elimination with partial pivoting
  const int n = m + 1;
  double a[33][34];
  double scale = 0.0;
  for (int i = 0; i < m; ++i) scale = std::max(scale, std::fabs(G[i * m + i]));
  if (!(scale > 0.0) || !std::isfinite(scale)) scale = 1.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= n; ++j) a[i][j] = 0.0;
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j < m; ++j) a[i][j] = G[i * m + j] / scale;
    a[i][m] = 1.0;
    a[m][i] = 1.0;
  }
  a[m][n] = 1.0;
  bool singular = false;
  for (int k = 0; k < n && !singular; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(a[i][k]) > std::fabs(a[p][k])) p = i;
    if (!(std::fabs(a[p][k]) > 1e-14)) {
      singular = true;
      break;
    }
    if (p != k)
      for (int j = 0; j <= n; ++j) std::swap(a[p][j], a[k][j]);
    for (int i = k + 1; i < n; ++i) {
      const double f = a[i][k] / a[k][k];
      for (int j = k; j <= n; ++j) a[i][j] -= f * a[k][j];
    }
  }
  double x[33];
  if (!singular) {
    for (int i = n - 1; i >= 0; --i) {
      double v = a[i][n];
      for (int j = i + 1; j < n; ++j) v -= a[i][j] * x[j];
      x[i] = v / a[i][i];
    }
    for (int i = 0; i < m; ++i) singular = singular || !std::isfinite(x[i]);
  }
  for (int i = 0; i < m; ++i) c[i] = singular ? (i == m - 1 ? 1.0 : 0.0) : x[i];
  return RIC_OK;
}

int ric_last_timings(const ric_ctx* ctx, double* ladder_ms, double* total_ms) {
  if (!ctx) return RIC_E_ARG;
  if (ladder_ms) *ladder_ms = ctx->ladder_ms;
  if (total_ms) *total_ms = ctx->total_ms;
  return RIC_OK;
}

const char* ric_last_error(const ric_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

}  // extern "C"
