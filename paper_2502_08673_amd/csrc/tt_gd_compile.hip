// tt_gd_compile.hip -- the GD sampler compiled for one circuit (host code).
//
// The interpreted sampler (tt_gd.hip) walks a gate program that it reads at
// run time, so a sample's probabilities and adjoints must live in memory and
// every gate waits for a load.  Here the same program -- Table 1's operators
// composed over each expression's Simplify form, the sigmoid embedding, the
// L2 loss, the chain rule through the operators, the GD update, hardening
// and the clause check -- is written out as straight-line device code for
// one circuit when the sampler is created, and compiled with the run-time
// compiler: every probability, adjoint and logit of a sample is a local
// value the compiler keeps in registers, one sample per thread.  Each gate
// turns into the same float expression the interpreter evaluates, in the
// same order.
#include <hip/hiprtc.h>

#include <cstdio>
#include <string>
#include <vector>

#include "tt_gd.h"

namespace tt {

namespace {

// Circuits above these sizes stay with the interpreter: the source (and its
// compile time) grows with the gates, and the registers with the slots.
constexpr size_t kCompiledMaxGates = 8192;
constexpr int kCompiledMaxSlots = 512;
constexpr size_t kCompiledMaxLits = 32768;

struct Writer {
  const GdProgram& P;
  std::string o;
  explicit Writer(const GdProgram& p) : P(p) {}

  void line(const std::string& s) {
    o += s;
    o += '\n';
  }
  static std::string num(int v) { return std::to_string(v); }
  // a float constant exactly as the interpreter holds it
  static std::string flt(float v) {
    char b[48];
    std::snprintf(b, sizeof(b), "%.9gf", (double)v);
    std::string s(b);
    if (s.find_first_of(".eEn") == std::string::npos) s.insert(s.size() - 1, ".0");
    return s;
  }
  bool is_var(int32_t slot) const { return slot < P.n_vslots; }
  std::string value(int32_t slot) const {
    return is_var(slot) ? "p" + num(slot) : "t" + num(slot - P.n_vslots);
  }
  std::string adjoint(int32_t slot) const {
    return is_var(slot) ? "g" + num(slot) : "a" + num(slot - P.n_vslots);
  }
  // an operand's value, 1 - p when negated (Table 1's NOT)
  std::string operand(int32_t o) const {
    const std::string v = value(o & kGdSlot);
    return (o & kGdNeg) ? "(1.f - " + v + ")" : v;
  }
  // Table 1: the operator's value at (x, y)
  std::string gate_value(const GdGate& g) const {
    if (g.op == TT_GATE_CONST) return flt((float)g.a);
    const std::string x = operand(g.a);
    if (g.op == TT_GATE_COPY) return x;
    const std::string y = operand(g.b);
    if (g.op == TT_GATE_AND) return x + " * " + y;
    if (g.op == TT_GATE_OR) return "1.f - (1.f - " + x + ") * (1.f - " + y + ")";
    if (g.op == TT_GATE_XOR) return "(1.f - " + x + ") * " + y + " + " + x + " * (1.f - " + y + ")";
    return x + " * " + y + " + (1.f - " + x + ") * (1.f - " + y + ")";
  }
  void forward(const GdGate& g) {
    const std::string z = gate_value(g);
    if (is_var(g.dst))
      line(value(g.dst) + " = " + z + ";");
    else
      line("const float " + value(g.dst) + " = " + z + ";");
  }
  // c added to an operand's adjoint (a negated operand takes -c)
  void give(int32_t o, const std::string& c) {
    line(adjoint(o & kGdSlot) + ((o & kGdNeg) ? " -= " : " += ") + c + ";");
  }
  // Table 1's derivatives times the gate's adjoint, to its operands
  void backward(const GdGate& g) {
    if (g.op == TT_GATE_CONST) return;
    const std::string adj = adjoint(g.dst);
    if (g.op == TT_GATE_COPY) {
      give(g.a, adj);
      return;
    }
    const std::string x = operand(g.a), y = operand(g.b);
    std::string dx, dy;
    if (g.op == TT_GATE_AND) {
      dx = y;
      dy = x;
    } else if (g.op == TT_GATE_OR) {
      dx = "(1.f - " + y + ")";
      dy = "(1.f - " + x + ")";
    } else if (g.op == TT_GATE_XOR) {
      dx = "(1.f - 2.f * " + y + ")";
      dy = "(1.f - 2.f * " + x + ")";
    } else {
      dx = "(2.f * " + y + " - 1.f)";
      dy = "(2.f * " + x + " - 1.f)";
    }
    give(g.a, adj + " * " + dx);
    give(g.b, adj + " * " + dy);
  }
  // zeroed adjoints of the temporaries that gates g0 .. g1 - 1 write
  void temp_adjoints(int g0, int g1) {
    for (int g = g0; g < g1; ++g)
      if (!is_var(P.gate[g].dst)) line("float " + adjoint(P.gate[g].dst) + " = 0.f;");
  }
};

}  // namespace

std::string gd_compiled_source(const GdProgram& P) {
  if (P.gate.size() > kCompiledMaxGates || P.n_vslots > kCompiledMaxSlots || P.lits.size() > kCompiledMaxLits)
    return std::string();
  Writer w(P);
  const int npi = P.n_pi, nv = P.n_vslots;
  const int n_iv = (int)P.iv_rng.size() - 1, n_aux = (int)P.aux_rng.size() - 1;
  // V0: the initial logits; V (may be V0, or null): the final ones.
  // primary (may be null): the first table of the distinct filter, where
  // every valid sample stores its index at its solution's place; table (may
  // be null): the filter's second table, cleared here
  w.line("extern \"C\" __global__ __launch_bounds__(256) void tt_gd_compiled(const float* V0, float* V, int batch, "
         "float lr, int iters, unsigned char* __restrict__ valid, unsigned long long* __restrict__ sol, "
         "int* __restrict__ primary, unsigned int pmask, int* __restrict__ table, unsigned int cap) {");
  w.line("const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;");
  w.line("if (table)");
  w.line("for (long t = s; t < (long)cap; t += (long)gridDim.x * blockDim.x) table[t] = -1;");
  w.line("if (s >= batch) return;");
  w.line("const float* V0r = V0 + s * " + Writer::num(npi) + "L;");
  for (int q = 0; q < npi; ++q) w.line("float v" + Writer::num(q) + " = V0r[" + Writer::num(q) + "];");
  // variables: primary inputs each step, constants as given, the rest from
  // their expressions
  for (int q = 0; q < nv; ++q) w.line("float p" + Writer::num(q) + " = " + Writer::flt(q < npi ? 0.f : P.cst[q]) + ";");
  w.line("for (int it = 0; it < iters; ++it) {");
  for (int q = 0; q < npi; ++q)
    w.line("p" + Writer::num(q) + " = 1.f / (1.f + __expf(-v" + Writer::num(q) + "));");
  for (int q = 0; q < nv; ++q) w.line("float g" + Writer::num(q) + " = 0.f;");
  // forward through the intermediate variables
  for (int x = 0; x < n_iv; ++x) {
    w.line("{");
    for (int g = P.iv_rng[x]; g < P.iv_rng[x + 1]; ++g) w.forward(P.gate[g]);
    w.line("}");
  }
  // loss: an auxiliary output's form must be 1, its adjoint 2 (P - 1) goes
  // back through its gates at once
  for (int x = 0; x < n_aux; ++x) {
    const int g0 = P.aux_rng[x], g1 = P.aux_rng[x + 1];
    w.line("{");
    for (int g = g0; g < g1; ++g) w.forward(P.gate[g]);
    w.temp_adjoints(g0, g1);
    const int32_t out = P.gate[g1 - 1].dst;
    w.line(w.adjoint(out) + " = 2.f * (" + w.value(out) + " - 1.f);");
    for (int g = g1 - 1; g >= g0; --g) w.backward(P.gate[g]);
    w.line("}");
  }
  // a constant on a primary input: (P - c)^2
  for (size_t i = 0; i + 1 < P.po.size(); i += 2)
    w.line("g" + Writer::num(P.po[i]) + " += 2.f * (p" + Writer::num(P.po[i]) + " - " +
           Writer::flt((float)P.po[i + 1]) + ");");
  // chain rule back through the intermediate variables, last first
  for (int x = n_iv - 1; x >= 0; --x) {
    const int g0 = P.iv_rng[x], g1 = P.iv_rng[x + 1];
    w.line("{");
    for (int g = g0; g < g1 - 1; ++g) w.forward(P.gate[g]);
    w.temp_adjoints(g0, g1);
    for (int g = g1 - 1; g >= g0; --g) w.backward(P.gate[g]);
    w.line("}");
  }
  for (int q = 0; q < npi; ++q) {
    const std::string n = Writer::num(q);
    w.line("v" + n + " -= lr * g" + n + " * p" + n + " * (1.f - p" + n + ");");
  }
  w.line("}");
  w.line("if (V) {");
  w.line("float* Vr = V + s * " + Writer::num(npi) + "L;");
  for (int q = 0; q < npi; ++q) w.line("Vr[" + Writer::num(q) + "] = v" + Writer::num(q) + ";");
  w.line("}");
  // harden: primary inputs from the logits' signs, the intermediate
  // variables through their gates on 0/1 values; check every clause
  for (int q = 0; q < npi; ++q) w.line("p" + Writer::num(q) + " = v" + Writer::num(q) + " > 0.f ? 1.f : 0.f;");
  for (int q = npi; q < nv; ++q) w.line("p" + Writer::num(q) + " = " + Writer::flt(P.cst[q]) + ";");
  for (int x = 0; x < n_iv; ++x) {
    w.line("{");
    for (int g = P.iv_rng[x]; g < P.iv_rng[x + 1]; ++g) w.forward(P.gate[g]);
    w.line("}");
  }
  w.line("bool ok = true;");
  for (size_t c = 0; c + 1 < P.coff.size(); ++c) {
    std::string any;
    for (int q = P.coff[c]; q < P.coff[c + 1]; ++q) {
      const int lit = P.lits[q];
      const std::string t = "(p" + Writer::num(lit >> 1) + " > 0.5f)";
      if (!any.empty()) any += " || ";
      any += (lit & 1) ? "!" + t : t;
    }
    w.line("ok = ok && (" + (any.empty() ? std::string("false") : any) + ");");
  }
  w.line("valid[s] = ok ? 1 : 0;");
  for (int wd = 0; wd < P.words; ++wd) {
    std::string bits = "0ull";
    for (int b = 0; b < 64 && 64 * wd + b < npi; ++b)
      bits += " | ((unsigned long long)(p" + Writer::num(64 * wd + b) + " > 0.5f) << " + Writer::num(b) + ")";
    w.line("const unsigned long long sw" + Writer::num(wd) + " = " + bits + ";");
    w.line("sol[s * " + Writer::num(P.words) + "L + " + Writer::num(wd) + "] = sw" + Writer::num(wd) + ";");
  }
  // the distinct filter's first pass: the same hash as the filter's
  w.line("if (primary && ok) {");
  w.line("unsigned long long h = " + std::to_string(kGdHashSeed) + "ull;");
  for (int wd = 0; wd < P.words; ++wd)
    w.line("h ^= sw" + Writer::num(wd) + "; h *= " + std::to_string(kGdHashMul) + "ull; h ^= h >> 31;");
  w.line("primary[(unsigned int)h & pmask] = (int)s;");
  w.line("}");
  w.line("}");
  return w.o;
}

int gd_compile(const GdProgram& P, hipModule_t* mod, hipFunction_t* fn) {
  *mod = nullptr;
  *fn = nullptr;
  const std::string src = gd_compiled_source(P);
  if (src.empty()) return -1;
  hiprtcProgram prog = nullptr;
  if (hiprtcCreateProgram(&prog, src.c_str(), "tt_gd_compiled.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    return -2;
  // as the library's own kernels: gfx950, no packed fp32 instructions
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops"};
  std::vector<char> code;
  hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
  size_t n = 0;
  if (r == HIPRTC_SUCCESS) r = hiprtcGetCodeSize(prog, &n);
  if (r == HIPRTC_SUCCESS) {
    code.resize(n);
    r = hiprtcGetCode(prog, code.data());
  }
  (void)hiprtcDestroyProgram(&prog);
  if (r != HIPRTC_SUCCESS || n == 0) return -3;
  hipModule_t m = nullptr;
  if (hipModuleLoadData(&m, code.data()) != hipSuccess) return -4;
  hipFunction_t f = nullptr;
  if (hipModuleGetFunction(&f, m, "tt_gd_compiled") != hipSuccess) {
    (void)hipModuleUnload(m);
    return -5;
  }
  *mod = m;
  *fn = f;
  return 0;
}

hipError_t launch_gd_compiled(hipFunction_t fn, const float* V0, float* V, int batch, float lr, int iters,
                              uint8_t* valid, uint64_t* sol, int32_t* primary, uint32_t primary_places,
                              int32_t* table, uint32_t cap, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  uint32_t pmask = primary_places ? primary_places - 1 : 0u;
  void* args[] = {&V0, &V, &batch, &lr, &iters, &valid, &sol, &primary, &pmask, &table, &cap};
  return hipModuleLaunchKernel(fn, (unsigned)((batch + 255) / 256), 1, 1, 256, 1, 1, 0, s, args, nullptr);
}

}  // namespace tt
