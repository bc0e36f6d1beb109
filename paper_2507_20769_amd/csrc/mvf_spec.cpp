// mvf_spec.cpp -- specialised forward-mode bounding kernels: generation of
// straight-line device code from a tape's compiled root programs, run-time
// compilation with hiprtc, an on-disk code-object cache, and the launch.
//
// What the generated kernel computes is exactly what the interpreter kernel
// computes (Sec. 3.1 Steps 1-3 with the mean value form of Sec. 2.2 and the
// tangent-mode interval gradient of Sec. 3.2): per root a point pass at the
// centre, tangent passes over the subdomain a chunk of gradient components at
// a time, MVF = [f(c)] + sum_i G_i (X_i - c_i) intersected with the NIE.  The
// generator walks the same instructions (with their constant-operand forms and
// slot-0 forwarding) and emits, per instruction, calls that give the results
// of the interpreter's calls for that opcode and operand kinds; slots become
// variables.  The decode, the dispatch and the slot-file moves disappear, and
// so does the arithmetic on structurally zero tangent components; facts known
// when generating (signs, degenerate and straddling factors) select cheaper
// forms of the same products and quotients.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cctype>
#include <dlfcn.h>
#include <chrono>
#include <cinttypes>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <sys/stat.h>
#include <utime.h>
#include <unistd.h>
#include <unordered_set>
#include <vector>

#include "mvf.h"
#include "mvf_internal.h"
#include "mvf_kernels.h"
#include "mvf_spec_internal.h"

namespace mvf {
namespace {

// the device headers the generated source includes (text embedded at build time)
#include "mvf_spec_headers.inc"

// instruction-passes: compile time grows about linearly (some 2 ms each on the
// GPU host; the 32-variable workload's adjoint, about 11,000, takes some 40 s,
// once: the code object is cached)
constexpr int64_t DEFAULT_MAX_CODE = 32000;
constexpr int SEGMENT = 32;                      // instructions per guarded block
constexpr int LDS_LEAD = 2;                      // statements a variable's LDS read runs ahead of its use
// Largest segment budget of the checkpointed adjoint.  Budgets up to 32 gave
// adjoints bitwise equal to the single-pass form on every workload measured
// (the 32-variable workload at 12, 24 and 32 over all 2^20 subdomains); at 40
// and at 58 that workload's objective came out different on the GPU although
// the generated code computes the same values (the host-side symbolic check
// of the generator agrees) and its mode switches pass the ISA check, so
// larger budgets are refused.  Both failing builds spill over a thousand
// VGPRs per lane.  For the same reason of an unexplained failure -- a memory
// fault of the batch workload's adjoint compiled for one wave per SIMD
// (segment budget 32, 64-lane workgroups) -- the adjoint kernels are not built
// for one wave per SIMD.
constexpr int MAX_CKPT_BUDGET = 32;
// Values recomputed at a segment's reload instead of stored: chains of at most
// this many cheap operations (sums, differences, products, squares, constant
// forms) from variables and constants.
constexpr int MAX_RELOAD_DEPTH = 2;
// A body line that only starts a new guarded block (segment boundaries of the
// checkpointed adjoint, so that a segment's checkpoint loads lead a block).
const char *const BLOCK_BREAK = "\x01";

struct Dec {
    uint32_t w0, op, ak, bk, a, b, d;
    double k;
};

Dec decode(const Instr &I) {
    Dec D;
    D.w0 = I.w0;
    D.op = I.w0 & 31u;
    D.ak = (I.w0 >> 5) & 3u;
    D.bk = (I.w0 >> 7) & 3u;
    D.a = I.w0 >> 16;
    D.b = I.w1 & 0xffffu;
    D.d = I.w1 >> 16;
    D.k = I.k;
    return D;
}

std::string lit(double x) {               // exact double literal
    char buf[64];
    std::snprintf(buf, sizeof buf, "%a", x);
    return buf;
}

// Tangent components that are structurally zero (the node does not depend on
// the component's variable) are carried as the literal kZero and cost nothing:
// a sum with zero is the other operand, a difference from zero its negation,
// and a product with zero is zero.  Where every enclosure involved is finite
// this is exactly the dense computation (endpoint products with zero are
// zeros; only the signs of zero endpoints may differ); a dense product of a
// zero component with an enclosure that is unbounded on both sides would be
// NaN where the exact derivative, zero, is kept here.
bool is_zero(const std::string &x) { return x == "kZero"; }
std::string add_tan(const std::string &x, const std::string &y) {
    if (is_zero(x)) return y;
    if (is_zero(y)) return x;
    return "iadd(" + x + ", " + y + ")";
}
std::string sub_tan(const std::string &x, const std::string &y) {
    if (is_zero(y)) return x;
    if (is_zero(x)) return "ineg(" + y + ")";
    return "isub(" + x + ", " + y + ")";
}
// f(x) for a product or scaling of x: zero stays zero
std::string scale_tan(const std::string &x, const std::string &pre, const std::string &post) {
    return is_zero(x) ? x : pre + x + post;
}

// Declarations of a generated function, each once (a recomputed segment
// assigns the variables of its first evaluation again).
struct Decls {
    std::vector<std::string> v;
    std::unordered_set<std::string> seen;
    void push_back(const std::string &d) {
        if (seen.insert(d).second) v.push_back(d);
    }
};

// The statements of one instruction (its tangent components, and a product's
// value) as trees of interval calls.  Products that do not depend on each
// other are emitted two at a time (imul2, imul_pos2: the two products in a
// row); the rest follow in dependence order.  Only the order of the
// instructions changes, not the arithmetic.
class Scheduler {
  public:
    Scheduler(std::string prefix, Decls &decl) : pre(std::move(prefix)), decl(decl) {}

    void add(const std::string &target, const std::string &expr) {
        size_t i = 0;
        roots.emplace_back(target, parse(expr, i));
    }

    std::string emit() {
        std::vector<int> depth(pool.size(), -1);
        int maxd = 0;
        for (const auto &r : roots) maxd = std::max(maxd, depth_of(r.second, depth));
        out.assign(pool.size(), "");
        for (const auto &r : roots)
            if (is_op(r.second)) out[r.second] = r.first;
        std::string s;
        for (int d = 1; d <= maxd; ++d) {
            int pend[2] = {-1, -1};                  // an unpaired imul, imul_pos
            for (size_t k = 0; k < pool.size(); ++k) {
                if (depth[k] != d || !is_op((int)k)) continue;
                const int kind = pool[k].fn == "imul" ? 0 : pool[k].fn == "imul_pos" ? 1 : -1;
                if (kind < 0) {
                    s += " " + name((int)k) + " = " + pool[k].fn + "(" + text(pool[k].args[0]) + ", " +
                         text(pool[k].args[1]) + ");";
                    continue;
                }
                if (pend[kind] < 0) {
                    pend[kind] = (int)k;
                    continue;
                }
                const Expr &a = pool[pend[kind]], &b = pool[k];
                s += std::string(" ") + (kind == 0 ? "imul2(" : "imul_pos2(") + text(a.args[0]) + ", " +
                     text(a.args[1]) + ", " + text(b.args[0]) + ", " + text(b.args[1]) + ", " + name(pend[kind]) +
                     ", " + name((int)k) + ");";
                pend[kind] = -1;
            }
            for (int kind = 0; kind < 2; ++kind)
                if (pend[kind] >= 0)
                    s += " " + name(pend[kind]) + " = " + pool[pend[kind]].fn + "(" + text(pool[pend[kind]].args[0]) +
                         ", " + text(pool[pend[kind]].args[1]) + ");";
        }
        for (const auto &r : roots)
            if (!is_op(r.second)) s += " " + r.first + " = " + text(r.second) + ";";
        return s;
    }

  private:
    struct Expr {
        std::string fn;                          // a scheduled call, or "" for a leaf
        std::string leaf;
        std::vector<int> args;
    };
    std::string pre;
    Decls &decl;
    std::vector<Expr> pool;
    std::vector<std::pair<std::string, int>> roots;
    std::vector<std::string> out;                 // result names of the emitted calls
    int n_tmp = 0;

    bool is_op(int k) const { return !pool[k].fn.empty() && pool[k].fn != "ineg"; }
    static bool scheduled(const std::string &f) {
        return f == "imul" || f == "imul_pos" || f == "iadd" || f == "isub" || f == "imulks" || f == "ineg";
    }
    static void skip(const std::string &e, size_t &i) {
        while (i < e.size() && e[i] == ' ') ++i;
    }
    int parse(const std::string &e, size_t &i) {
        skip(e, i);
        const size_t start = i;
        size_t j = i;
        while (j < e.size() && (std::isalnum((unsigned char)e[j]) || e[j] == '_')) ++j;
        if (j < e.size() && e[j] == '(' && scheduled(e.substr(i, j - i))) {
            Expr x;
            x.fn = e.substr(i, j - i);
            i = j + 1;
            for (;;) {
                x.args.push_back(parse(e, i));
                skip(e, i);
                if (e[i++] == ')') break;        // else ','
            }
            pool.push_back(x);
            return (int)pool.size() - 1;
        }
        int dep = 0;                             // a leaf: up to a ',' or ')' outside brackets
        for (i = start; i < e.size(); ++i) {
            const char c = e[i];
            if (c == '(' || c == '{') ++dep;
            else if ((c == ')' || c == '}') && dep > 0) --dep;
            else if (dep == 0 && (c == ',' || c == ')')) break;
        }
        size_t end = i;
        while (end > start && e[end - 1] == ' ') --end;
        Expr x;
        x.leaf = e.substr(start, end - start);
        pool.push_back(x);
        return (int)pool.size() - 1;
    }
    int depth_of(int k, std::vector<int> &depth) {
        if (depth[k] >= 0) return depth[k];
        int d = 0;
        for (int a : pool[k].args) d = std::max(d, depth_of(a, depth));
        return depth[k] = pool[k].fn.empty() ? 0 : pool[k].fn == "ineg" ? d : d + 1;
    }
    std::string name(int k) {
        if (out[k].empty()) {
            out[k] = pre + std::to_string(n_tmp++);
            decl.push_back("Iv " + out[k] + ";");
        }
        return out[k];
    }
    std::string text(int k) {
        if (pool[k].fn.empty()) return pool[k].leaf;
        if (pool[k].fn == "ineg") return "ineg(" + text(pool[k].args[0]) + ")";
        return name(k);
    }
};

// Segments of one root program for the checkpointed adjoint: start[j] are
// program-relative boundaries (start[0] = 0, start[K] = len); in[j] are the
// instructions (absolute) whose values segment j reads from before it.  The
// value pass stores each such value once, at the first boundary j in
// 1 .. K-2 whose segment reads it (store[j]), at checkpoint index slot[pc];
// a value that one cheap operation makes from variables and constants alone
// (again[pc - begin]) is not stored but recomputed where a segment reloads
// it (the same operation on the same operands: the same bits, no traffic).
// ck_count intervals per lane in all.
struct SegPlan {
    std::vector<int> pa, pb;                     // producers of an instruction's slot operands (or -1)
    std::vector<int> start;
    std::vector<std::vector<int>> in;
    std::vector<std::vector<int>> store;
    std::map<int, int> slot;
    std::vector<char> again;
    int ck_count = 0;
};

// A cheap operation (no division, root or transcendental), slot operands allowed.
bool cheap_op(const Dec &I) {
    switch (I.op) {
    case I_ADD: case I_SUB: case I_MUL: case I_SQR: case I_ADDK: case I_KSUB: case I_MULK: case I_MULKN:
        return true;
    default:
        return false;
    }
}

// One cheap operation on variables and constants: the first step of a value
// recomputed at reload instead of checkpointed (chains of MAX_RELOAD_DEPTH).
bool recompute_at_reload(const Dec &I) {
    switch (I.op) {
    case I_ADD: case I_SUB: case I_MUL:
        return I.ak != K_SLOT && I.bk != K_SLOT;
    case I_SQR: case I_ADDK: case I_KSUB: case I_LOAD: case I_MULK: case I_MULKN:
        return I.ak != K_SLOT;
    default:
        return false;
    }
}

// One pass over one root program.  C == 0: values only, variables at the
// centre (point) or over the subdomain; C > 0: values and the tangent
// components [c0, c0 + C).  With tape (C == 0 over the subdomain) the value
// pass also computes the local partials the reverse sweep needs (those the
// interpreter writes to its record tape), and reverse() then emits the sweep;
// adjoint() emits the checkpointed form of both.
class PassWriter {
  public:
    PassWriter(const Compiled &Cp, int root, int C, int c0, bool point, bool tape = false, int gl = 0)
        : P(Cp), r(root), C(C), c0(c0), point(point), partials(tape), lead(!tape), gl_base(Cp.n_vars - gl) {}

    // body lines (declarations first, then guarded blocks) and the names of
    // the result's value and components
    void emit(Decls &decl, std::vector<std::string> &body, std::string &val, std::vector<std::string> &tan) {
        const RootProg &rp = P.roots[r];
        reset_slots();
        for (int pc = rp.begin; pc < rp.begin + rp.len; ++pc) instr(pc, decl, body);
        const int rs = rp.result_slot;
        val = slot_val.at(rs);
        tan = slot_tan.at(rs);
    }

    // One pass over the union of the root cones, every node once.  Right after
    // the instruction that computes root q, what root q's bound takes from this
    // pass is written out, so that no root stays live to the end: its value at
    // the centre (point pass), its value (value pass), or its value and this
    // pass's gradient components folded into its mean value form (tangent
    // pass; components in index order, structurally zero ones skipped).
    void emit_union(Decls &decl, std::vector<std::string> &body) {
        const RootProg &up = P.uprog;
        std::map<uint32_t, int> last_write;              // slot -> the last instruction writing it
        for (int pc = up.begin; pc < up.begin + up.len; ++pc) last_write[decode(P.instr[pc]).d] = pc;
        std::map<int, std::vector<int>> defs;            // instruction -> the roots it computes
        for (int q = 0; q < (int)P.union_slots.size(); ++q)
            defs[last_write.at((uint32_t)P.union_slots[q])].push_back(q);
        reset_slots();
        for (int pc = up.begin; pc < up.begin + up.len; ++pc) {
            instr(pc, decl, body);
            const auto it = defs.find(pc);
            if (it == defs.end()) continue;
            const uint32_t d = decode(P.instr[pc]).d;
            for (int q : it->second) body.push_back(root_out(q, slot_val.at(d), slot_tan.at(d)));
        }
    }
    std::string root_out(int q, const std::string &val, const std::vector<std::string> &tan) const {
        const std::string Q = std::to_string(q);
        if (C == 0) return std::string(point ? "FC[" : "V[") + Q + "] = " + val + ";";
        std::string s = "{ ";
        if (c0 == 0) s += "nie[" + Q + "] = " + val + "; ";
        for (int t = 0; t < C; ++t)
            if (!is_zero(tan[t]))
                s += "const Iv d" + std::to_string(t) + " = spec_dx(L, " + std::to_string(c0 + t) + "); ";
        for (int t = 0; t < C; ++t)
            if (!is_zero(tan[t]))
                s += "acc[" + Q + "] = iadd(acc[" + Q + "], imul_dx(" + tan[t] + ", d" + std::to_string(t) + ")); ";
        return s + "}";
    }

    // The reverse sweep after emit() with tape: the root's adjoint is [1, 1],
    // instructions in reverse order, each contribution to a slot operand
    // written at the operand's last use (its init flag) and accumulated
    // otherwise, contributions to variables accumulated into G[i] in sweep
    // order (the interpreter's reverse_sweep, with records read from the
    // value pass's variables).
    void reverse(Decls &decl, std::vector<std::string> &body) {
        const RootProg &rp = P.roots[r];
        body.push_back("y" + std::to_string(slot_prod.at(rp.result_slot)) + " = kOne;");
        sweep(decl, body, rp.begin, rp.begin + rp.len);
    }

    // Value pass and reverse sweep with checkpointed recomputation.  The
    // program is cut into segments [start[j], start[j+1]).  A value-only pass
    // runs segments 0 .. K-2 and stores at each boundary start[j] (j >= 1)
    // the values produced before it that segment j reads and no earlier
    // boundary stored (to the checkpoint buffer, one index per value).
    // Segment K-1 then runs with its local partials and is swept at once;
    // every earlier segment, last first, reloads its inputs (cheap values of
    // variables and constants alone are recomputed instead), runs again with
    // its partials and is swept.  The
    // adjoints of values that cross a boundary stay in variables.  The
    // recomputation repeats the same operations on the same operands, so the
    // result is bitwise that of reverse() after a single value pass; domain
    // tests are made once, in the first pass.  Writes the NIE value to nie.
    void adjoint(Decls &decl, std::vector<std::string> &body, const SegPlan &S) {
        const std::vector<int> &start = S.start;
        const std::vector<std::vector<int>> &in = S.in;
        const RootProg &rp = P.roots[r];
        const int K = (int)start.size() - 1;
        reset_slots();
        std::vector<Snapshot> snap(K);
        partials = false;
        for (int j = 0; j + 1 < K; ++j) {
            if (j >= 1) {
                body.push_back(BLOCK_BREAK);
                std::string st;
                for (int p : S.store[j])
                    st += "spec_ck_st(L, " + std::to_string(S.slot.at(p)) + ", v" + std::to_string(p) + "); ";
                body.push_back(st);
            }
            snap[j] = save();
            for (int pc = rp.begin + start[j]; pc < rp.begin + start[j + 1]; ++pc) instr(pc, decl, body);
        }
        // the checkpoint loads of segment j and its recomputed inputs
        auto loads_of = [&](int j) {
            std::string ld;
            for (int p : in[j])
                if (!S.again[p - rp.begin])
                    ld += "v" + std::to_string(p) + " = spec_ck_ld(L, " + std::to_string(S.slot.at(p)) + "); ";
            return ld;
        };
        // recomputed inputs, each after the recomputed values it reads (program order)
        auto recomputed_of = [&](int j) {
            std::set<int> need;
            std::vector<int> todo;
            for (int p : in[j])
                if (S.again[p - rp.begin]) todo.push_back(p);
            while (!todo.empty()) {
                const int p = todo.back();
                todo.pop_back();
                if (!need.insert(p).second) continue;
                for (int q : {S.pa[p - rp.begin], S.pb[p - rp.begin]})
                    if (q >= 0) todo.push_back(q);
            }
            std::string re;
            for (int p : need) re += value_stmt.at(p);
            return re;
        };
        partials = true;
        for (int pc = rp.begin + start[K - 1]; pc < rp.begin + start[K]; ++pc) instr(pc, decl, body);
        decl.push_back("Iv nie;");
        body.push_back("nie = " + slot_val.at(rp.result_slot) + ";");
        body.push_back(zero_gradient());
        body.push_back("y" + std::to_string(slot_prod.at(rp.result_slot)) + " = kOne;");
        sweep(decl, body, rp.begin + start[K - 1], rp.begin + start[K]);
        checks = false;
        for (int j = K - 2; j >= 0; --j) {
            restore(snap[j]);
            body.push_back(BLOCK_BREAK);
            // loads issued at the segment's start: issued a segment earlier, into registers they
            // held through the previous segment's sweep (1.7x slower on the batch workload), into
            // LDS by the memory system (global_load_lds) they still ran 1.2-1.5x slower
            if (j >= 1) body.push_back(loads_of(j) + recomputed_of(j));
            for (int pc = rp.begin + start[j]; pc < rp.begin + start[j + 1]; ++pc) instr(pc, decl, body);
            sweep(decl, body, rp.begin + start[j], rp.begin + start[j + 1]);
        }
        checks = true;
    }


    std::string zero_gradient() const {
        std::string s;
        for (int i = 0; i < P.n_vars; ++i) s += grad_ref(i) + " = kZero; ";
        return s;
    }
    // gradient component i: a register, or its LDS entry
    std::string grad_ref(int i) const {
        return i < gl_base ? "G[" + std::to_string(i) + "]" : "spec_gl(L, " + std::to_string(i - gl_base) + ")";
    }
    // the LDS-resident components copied into the register array the caller combines
    std::string gradient_out() const {
        std::string s;
        for (int i = gl_base; i < P.n_vars; ++i) s += "G[" + std::to_string(i) + "] = " + grad_ref(i) + "; ";
        return s;
    }

  private:
    // sweep instructions [lo, hi) in reverse order (their steps recorded by
    // the last pass with partials over them)
    void sweep(Decls &decl, std::vector<std::string> &body, int lo, int hi) {
        for (int pc = lo; pc < hi; ++pc) decl.push_back("Iv y" + std::to_string(pc) + ";");
        for (int pcs = hi - 1; pcs >= lo; --pcs) {
            const auto it = steps.find(pcs);
            if (it == steps.end()) continue;
            const Step &st = it->second;
            const Dec &I = st.I;
            const std::string pc = std::to_string(st.pc), zb = "y" + pc;
            const bool ia = (I.w0 & W0_INIT_A) != 0, ib = (I.w0 & W0_INIT_B) != 0;
            std::string s;
            auto contribute = [&](uint32_t kind, uint32_t a, int prod, bool init, bool neg, const std::string &c) {
                if (kind == K_SLOT) {
                    const std::string y = "y" + std::to_string(prod);
                    if (init) s += y + " = " + (neg ? "ineg(" + c + ")" : c) + "; ";
                    else s += y + " = " + (neg ? "isub(" : "iadd(") + y + ", " + c + "); ";
                } else if (kind == K_VAR) {
                    const std::string g = grad_ref((int)a);
                    s += g + " = " + (neg ? "isub(" : "iadd(") + g + ", " + c + "); ";
                }
            };
            switch (I.op) {
            case I_ADD:
            case I_SUB:
                contribute(I.ak, I.a, st.pa, ia, false, zb);
                contribute(I.bk, I.b, st.pb, ib, I.op == I_SUB, zb);
                break;
            case I_MUL:
                if (I.ak != K_CONST && I.bk != K_CONST && st.nv == st.nu) {
                    // both products at once (the same operations, interleaved)
                    const std::string P = "pa" + pc, Q = "pb" + pc;
                    decl.push_back("Iv " + P + ";");
                    decl.push_back("Iv " + Q + ";");
                    s += std::string(st.nv ? "imul_pos2(" : "imul2(") + zb + ", " + st.V + ", " + zb + ", " + st.U +
                         ", " + P + ", " + Q + "); ";
                    contribute(I.ak, I.a, st.pa, ia, false, P);
                    contribute(I.bk, I.b, st.pb, ib, false, Q);
                    break;
                }
                if (I.ak != K_CONST) contribute(I.ak, I.a, st.pa, ia, false, mul_by(zb, st.V, st.nv, false));
                if (I.bk != K_CONST) contribute(I.bk, I.b, st.pb, ib, false, mul_by(zb, st.U, st.nu, false));
                break;
            case I_DIV: {
                const std::string T = "t" + pc;
                decl.push_back("Iv " + T + ";");
                s += T + " = " + mul_by(zb, "r" + pc, st.nv, false) + "; ";
                contribute(I.ak, I.a, st.pa, ia, false, T);
                if (I.bk != K_CONST) contribute(I.bk, I.b, st.pb, ib, true, mul_by(T, "v" + pc, st.nz, false));
                break;
            }
            case I_SQR:
            case I_SQRT:
            case I_EXP:
            case I_LOG:
            case I_TANH:
            case I_SIN:
            case I_COS:
                if (I.ak != K_CONST)
                    contribute(I.ak, I.a, st.pa, ia, false, mul_by(zb, "q" + pc, nonneg_deriv(I, st.nu), false));
                break;
            case I_ADDK:
            case I_KSUB:
            case I_LOAD:
                contribute(I.ak, I.a, st.pa, ia, I.op == I_KSUB, zb);
                break;
            case I_MULK:
            case I_MULKN:
                contribute(I.ak, I.a, st.pa, ia, false,
                           "imulks(" + (I.op == I_MULKN ? "ineg(" + zb + ")" : zb) + ", " + lit(I.k) + ")");
                break;
            default:   // I_DIVK, I_DIVKN
                contribute(I.ak, I.a, st.pa, ia, false,
                           "imul_pos(" + (I.op == I_DIVKN ? "ineg(" + zb + ")" : zb) + ", " + st.aux + ")");
                break;
            }
            body.push_back(s);
        }
    }

    const Compiled &P;
    int r, C, c0;
    bool point;
    bool partials;                               // compute the local partials (and record the steps)
    const bool lead;                             // place variable reads LDS_LEAD statements early
    const int gl_base;                           // gradient components from here on live in LDS
    std::map<int, std::string> value_stmt;       // value-pass statements, for recomputation at reload
    int n_hoist = 0;
    bool checks = true;                          // emit the domain tests
    std::vector<std::string> slot_val;
    std::vector<std::vector<std::string>> slot_tan;
    std::vector<int> slot_prod;                  // instruction that wrote the slot's current value
    std::vector<char> slot_nn;                   // the slot's value is nonnegative (see nonneg_result)
    struct Step {
        int pc;
        Dec I;
        std::string U, V, aux;                   // operand value expressions; 1/k enclosure of a DIVK
        int pa, pb;                              // producers of slot operands
        bool nu, nv, nz;                         // operands and result known nonnegative
    };
    std::map<int, Step> steps;                   // by instruction, from the last pass with partials
    struct Snapshot {
        std::vector<std::string> val;
        std::vector<int> prod;
        std::vector<char> nn;
    };

    // the root's program, or the union of the root cones for r = number of roots
    const RootProg &prog() const { return r < (int)P.roots.size() ? P.roots[r] : P.uprog; }

    void reset_slots() {
        const RootProg &rp = prog();
        slot_val.assign(std::max(rp.n_slots, 1) + 1, "");
        slot_tan.assign(slot_val.size(), std::vector<std::string>());
        slot_prod.assign(slot_val.size(), -1);
        slot_nn.assign(slot_val.size(), 0);
    }
    Snapshot save() const { return Snapshot{slot_val, slot_prod, slot_nn}; }
    void restore(const Snapshot &S) {
        slot_val = S.val;
        slot_prod = S.prod;
        slot_nn = S.nn;
        slot_tan.assign(slot_val.size(), std::vector<std::string>());
    }

    void ensure(size_t s) {
        if (s >= slot_val.size()) {
            slot_val.resize(s + 1);
            slot_tan.resize(s + 1);
            slot_prod.resize(s + 1, -1);
            slot_nn.resize(s + 1, 0);
        }
    }

    // Sign facts known at generation time.  A value is "nonnegative" when every
    // enclosure of it has lo >= 0 on every subdomain whose bounds are kept: a
    // subdomain where a domain test fails (a denominator enclosing 0, a sqrt or
    // log argument below 0) is flagged and its bounds are discarded.
    bool nonneg(uint32_t kind, uint32_t a, double k) const {
        if (kind == K_SLOT) return a < slot_nn.size() && slot_nn[a];
        if (kind == K_CONST) return k >= 0.0;
        return false;
    }
    static bool nonneg_result(const Dec &I, bool nu, bool nv) {
        switch (I.op) {
        case I_ADD: case I_MUL: case I_DIV: return nu && nv;
        case I_SQR: case I_SQRT: case I_EXP: return true;
        case I_ADDK: case I_MULK: return nu && I.k >= 0.0;
        case I_DIVK: return nu;                   // k > 0
        case I_LOAD: return nu;
        default: return false;
        }
    }
    // the derivative factor of a unary op is nonnegative where the bounds are kept
    static bool nonneg_deriv(const Dec &I, bool nu) {
        return I.op == I_SQRT || I.op == I_EXP || I.op == I_LOG || I.op == I_TANH || (I.op == I_SQR && nu);
    }
    // U * R, one-sided when R is known nonnegative (the extreme products then
    // come from U's endpoints alone: the same result up to the signs of zeros)
    static std::string mul_by(const std::string &u, const std::string &r, bool r_nn, bool r_first = true) {
        if (r_nn) return "imul_pos(" + u + ", " + r + ")";
        return r_first ? "imul(" + r + ", " + u + ")" : "imul(" + u + ", " + r + ")";
    }

    static std::string aux_literal(const Instr &aux) {
        uint64_t bits = (uint64_t)aux.w1 << 32 | aux.w0;
        double rlo;
        std::memcpy(&rlo, &bits, 8);
        return "Iv{" + lit(rlo) + ", " + lit(aux.k) + "}";
    }

    // operand: value expression; components (dense), or the hit component of
    // a variable (-1 otherwise)
    void fetch(uint32_t kind, uint32_t a, double k, std::string &v, std::vector<std::string> &t, bool &dense,
               int &hit) {
        dense = false;
        hit = -1;
        t.clear();
        if (kind == K_SLOT) {
            ensure(a);
            v = slot_val[a];
            t = slot_tan[a];
            dense = true;
        } else if (kind == K_VAR) {
            v = std::string(point ? "spec_c(L, " : "spec_x(L, ") + std::to_string(a) + ")";
            const int h = (int)a - c0;
            hit = h >= 0 && h < C ? h : -1;
        } else {
            v = "Iv{" + lit(k) + ", " + lit(-k) + "}";
        }
    }

    // A variable's LDS read placed LDS_LEAD statements ahead of its use, into a
    // temporary, so that its latency overlaps the arithmetic in between (the
    // compiler keeps reads next to their uses under this register pressure).
    // Tangent-mode and point passes only: in the adjoint's value pass the
    // longer live ranges cost more spills than the overlap gains.
    std::string hoist(const std::string &e, Decls &decl, std::vector<std::string> &body) {
        const std::string name = "x" + std::to_string(r) + (point ? "p" : "t") + std::to_string(c0) + "_" +
                                 std::to_string(n_hoist++);
        decl.push_back("Iv " + name + ";");
        const size_t d = (size_t)LDS_LEAD;
        const size_t pos = body.size() > d ? body.size() - d : 0;
        body.insert(body.begin() + (long)pos, name + " = " + e + ";");
        return name;
    }

    void instr(int pc, Decls &decl, std::vector<std::string> &body) {
        const Dec I = decode(P.instr[pc]);
        std::string U, V;
        std::vector<std::string> A, B;
        bool ad = false, bd = false;
        int ha = -1, hb = -1;
        fetch(I.ak, I.a, I.k, U, A, ad, ha);
        if (I.op <= I_DIV) fetch(I.bk, I.b, I.k, V, B, bd, hb);
        const std::string Ue = U, Ve = V;                // operand expressions for the sweep
        if (lead && LDS_LEAD > 0) {
            if (I.ak == K_VAR) U = hoist(U, decl, body);
            if (I.op <= I_DIV && I.bk == K_VAR) V = I.ak == K_VAR && I.a == I.b ? U : hoist(V, decl, body);
        }
        const bool nu = nonneg(I.ak, I.a, I.k), nv = I.op <= I_DIV && nonneg(I.bk, I.b, I.k);
        const bool nz = nonneg_result(I, nu, nv);
        if (partials) {
            Step st{pc, I, Ue, Ve, "", I.ak == K_SLOT ? slot_prod.at(I.a) : -1,
                    I.op <= I_DIV && I.bk == K_SLOT ? slot_prod.at(I.b) : -1, nu, nv, nz};
            if (I.op == I_DIVK || I.op == I_DIVKN) st.aux = aux_literal(P.instr.at(I.b));
            steps[pc] = st;
        }
        const std::string z = "v" + std::to_string(pc);
        std::string s;                                   // the statements of this instruction
        std::vector<std::string> Z(C, "kZero");
        std::string zexpr;                               // a product's value, scheduled with the components
        auto hit_add = [&](int h, const std::string &x) { if (h >= 0) Z[h] = add_tan(Z[h], x); };
        auto hit_sub = [&](int h, const std::string &x) { if (h >= 0) Z[h] = sub_tan(Z[h], x); };
        const std::string k = lit(I.k);
        switch (I.op) {
        case I_ADD:
        case I_SUB: {
            const bool add = I.op == I_ADD;
            s += z + " = " + (add ? "iadd(" : "isub(") + U + ", " + V + ");";
            if (ad) for (int t = 0; t < C; ++t) Z[t] = A[t];
            if (bd) for (int t = 0; t < C; ++t) Z[t] = add ? add_tan(Z[t], B[t]) : sub_tan(Z[t], B[t]);
            hit_add(ha, "kOne");
            if (add) hit_add(hb, "kOne");
            else hit_sub(hb, "kOne");
            break;
        }
        case I_MUL:
            if (point && (I.ak == K_VAR || I.bk == K_VAR))     // a variable at the centre is degenerate
                zexpr = I.bk == K_VAR ? "imul_deg(" + U + ", " + V + ")" : "imul_deg(" + V + ", " + U + ")";
            else
                zexpr = nv ? mul_by(U, V, true) : nu ? mul_by(V, U, true) : "imul(" + U + ", " + V + ")";
            if (ad) for (int t = 0; t < C; ++t) Z[t] = is_zero(A[t]) ? A[t] : mul_by(A[t], V, nv);
            if (bd) for (int t = 0; t < C; ++t) Z[t] = add_tan(Z[t], is_zero(B[t]) ? B[t] : mul_by(B[t], U, nu));
            hit_add(ha, V);
            hit_add(hb, U);
            break;
        case I_DIV: {
            const std::string tv = "b" + std::to_string(pc);
            decl.push_back("Iv " + tv + ";");
            s += tv + " = " + V + "; ";
            if (checks) s += "bad |= (" + tv + ".lo <= 0.0 && " + tv + ".nh <= 0.0) ? 1u : 0u; ";
            s += z + " = " + (nv ? "idiv_pos(" : "idiv(") + U + ", " + tv + ");";
            if (C > 0 || partials) {
                const std::string R = "r" + std::to_string(pc);
                decl.push_back("Iv " + R + ";");
                s += " " + R + " = " + (nv ? "irecip_pos(" : "irecip(") + tv + ");";
            }
            if (C > 0) {
                const std::string R = "r" + std::to_string(pc);
                if (ad) for (int t = 0; t < C; ++t) Z[t] = A[t];
                if (bd)
                    for (int t = 0; t < C; ++t) Z[t] = sub_tan(Z[t], is_zero(B[t]) ? B[t] : mul_by(B[t], z, nz));
                hit_add(ha, "kOne");
                hit_sub(hb, z);
                for (int t = 0; t < C; ++t) Z[t] = is_zero(Z[t]) ? Z[t] : mul_by(Z[t], R, nv, false);
            }
            break;
        }
        case I_SQR:
        case I_SQRT:
        case I_EXP:
        case I_LOG:
        case I_TANH:
        case I_SIN:
        case I_COS: {
            const std::string tu = "u" + std::to_string(pc), D = "q" + std::to_string(pc);
            decl.push_back("Iv " + tu + ";");
            s += tu + " = " + U + "; ";
            std::string dexpr;
            if (I.op == I_SQR) {
                s += z + " = " + (point && I.ak == K_VAR ? "isqr_deg(" : "isqr(") + tu + ");";
                dexpr = "itwice(" + tu + ")";
            } else if (I.op == I_SQRT) {
                if (checks) s += "bad |= " + tu + ".lo < 0.0 ? 1u : 0u; ";
                s += z + " = isqrt(" + tu + ");";
                dexpr = "isqrt_deriv(" + z + ")";
            } else if (I.op == I_EXP) {
                s += z + " = iexp(" + tu + ");";
                dexpr = z;
            } else if (I.op == I_LOG) {
                if (checks) s += "bad |= " + tu + ".lo <= 0.0 ? 1u : 0u; ";
                s += z + " = ilog(" + tu + ");";
                dexpr = "irecip_pos(" + tu + ")";         // u > 0 wherever the bounds are kept
            } else if (I.op == I_TANH) {
                s += z + " = itanh(" + tu + ");";
                dexpr = "itanh_deriv(" + z + ")";
            } else if (I.op == I_SIN) {
                s += z + " = isin(" + tu + ");";
                dexpr = "isin_deriv(" + tu + ")";
            } else {
                s += z + " = icos(" + tu + ");";
                dexpr = "icos_deriv(" + tu + ")";
            }
            if (C > 0 || partials) {
                decl.push_back("Iv " + D + ";");
                s += " " + D + " = " + dexpr + ";";
            }
            if (C > 0) {
                const bool dn = nonneg_deriv(I, nu);
                if (ad) for (int t = 0; t < C; ++t) Z[t] = is_zero(A[t]) ? A[t] : mul_by(A[t], D, dn);
                if (ha >= 0) Z[ha] = D;
            }
            break;
        }
        case I_ADDK:
        case I_KSUB:
        case I_LOAD: {
            const bool ks = I.op == I_KSUB;
            const std::string tu = "u" + std::to_string(pc);
            decl.push_back("Iv " + tu + ";");
            s += tu + " = " + U + "; ";
            if (I.op == I_ADDK) s += z + " = iaddk(" + tu + ", " + k + ");";
            else if (ks) s += z + " = iksub(" + k + ", " + tu + ");";
            else s += z + " = " + tu + ";";
            if (ad) for (int t = 0; t < C; ++t) Z[t] = ks ? scale_tan(A[t], "ineg(", ")") : A[t];
            if (ha >= 0) Z[ha] = ks ? "ineg(kOne)" : "kOne";
            break;
        }
        case I_MULK:
        case I_MULKN: {
            const bool ng = I.op == I_MULKN;
            auto sg = [&](const std::string &x) { return ng ? "ineg(" + x + ")" : x; };
            s += z + " = imulks(" + sg(U) + ", " + k + ");";
            if (ad) for (int t = 0; t < C; ++t) Z[t] = is_zero(A[t]) ? A[t] : "imulks(" + sg(A[t]) + ", " + k + ")";
            if (ha >= 0) Z[ha] = "imulks(" + sg("kOne") + ", " + k + ")";
            break;
        }
        default: {   // I_DIVK, I_DIVKN: operand b indexes the enclosure of 1/k
            const bool ng = I.op == I_DIVKN;
            auto sg = [&](const std::string &x) { return ng ? "ineg(" + x + ")" : x; };
            s += z + " = idivk(" + sg(U) + ", " + k + ");";
            if (C > 0) {
                const std::string R = aux_literal(P.instr.at(I.b));
                if (ad) for (int t = 0; t < C; ++t) Z[t] = is_zero(A[t]) ? A[t] : "imul_pos(" + sg(A[t]) + ", " + R + ")";
                if (ha >= 0) Z[ha] = "imul_pos(" + sg("kOne") + ", " + R + ")";
            }
            break;
        }
        }
        decl.push_back("Iv " + z + ";");
        std::vector<std::string> tn(C);
        Scheduler sch("h" + std::to_string(pc) + "_", decl);
        if (!zexpr.empty()) sch.add(z, zexpr);
        for (int t = 0; t < C; ++t) {
            if (is_zero(Z[t])) {
                tn[t] = Z[t];
                continue;
            }
            tn[t] = "g" + std::to_string(pc) + "_" + std::to_string(t);
            decl.push_back("Iv " + tn[t] + ";");
            sch.add(tn[t], Z[t]);
        }
        s += sch.emit();
        if (!partials && C == 0) value_stmt[pc] = s;
        body.push_back(s);
        ensure(I.d);
        slot_val[I.d] = z;
        slot_tan[I.d] = tn;
        slot_prod[I.d] = pc;
        slot_nn[I.d] = nz;
    }
};

void write_guarded(std::string &out, const std::vector<std::string> &body) {
    size_t in_block = 0;
    for (const auto &line : body) {
        if (line == BLOCK_BREAK) {
            if (in_block) out += "    }\n";
            in_block = 0;
            continue;
        }
        if (in_block == 0) out += "    if (go) {\n";
        out += "        " + line + "\n";
        if (++in_block == (size_t)SEGMENT) {
            out += "    }\n";
            in_block = 0;
        }
    }
    if (in_block) out += "    }\n";
}

// A segment fits the budget when its inputs from earlier segments plus the
// values and local partials it computes (an estimate of what its
// recomputation and sweep keep in registers) stay within budget intervals.
// budget <= 0: one segment (no recomputation).
SegPlan plan_segments(const Compiled &P, int r, int budget) {
    const RootProg &rp = P.roots[r];
    const int len = rp.len;
    std::vector<int> pa(len, -1), pb(len, -1), cost(len, 1);
    std::vector<int> prod(std::max(rp.n_slots, 1) + 1, -1);
    SegPlan S;
    S.again.assign(len, 0);
    std::vector<int> depth(len, 0);                // cheap operations from variables and constants
    for (int i = 0; i < len; ++i) {
        const Dec I = decode(P.instr[rp.begin + i]);
        if (I.ak == K_SLOT && I.a < prod.size()) pa[i] = prod[I.a];
        if (I.op <= I_DIV && I.bk == K_SLOT && I.b < prod.size()) pb[i] = prod[I.b];
        if (recompute_at_reload(I)) {
            depth[i] = 1;
        } else if (cheap_op(I)) {
            int d = 0;
            for (int p : {pa[i], pb[i]})
                if (p >= 0) d = std::max(d, depth[p - rp.begin] > 0 ? depth[p - rp.begin] : MAX_RELOAD_DEPTH);
            if ((I.ak != K_SLOT || pa[i] >= 0) && (I.op > I_DIV || I.bk != K_SLOT || pb[i] >= 0)) depth[i] = d + 1;
        }
        S.again[i] = depth[i] > 0 && depth[i] <= MAX_RELOAD_DEPTH;
        if (I.op == I_DIV || (is_unary_fn(I.op) && I.op != I_EXP)) cost[i] = 2;     // 1/V, or the derivative
        if (I.d >= prod.size()) prod.resize(I.d + 1, -1);
        prod[I.d] = rp.begin + i;
    }
    S.start.push_back(0);
    if (budget <= 0) {
        S.start.push_back(len);
    } else {
        // The cut points with the fewest checkpoint intervals in all (the inputs
        // of every segment but the first, which reads only variables and
        // constants, and the last, which runs while its inputs are still in
        // registers), every segment within budget, fewer segments on ties:
        // a shortest path over the cut positions.  Where the live set across
        // a cut dips, cutting there saves the difference at every boundary
        // (about 11 % of the checkpoints of the random DAG workloads against
        // cutting greedily at the budget).
        const int64_t INF = INT64_MAX / 4;
        std::vector<int64_t> best(len + 1, INF);      // checkpoints * 2^20 + segments
        std::vector<int> from(len + 1, -1);
        best[0] = 0;
        std::vector<int> inset;
        for (int s = 0; s < len; ++s) {
            if (best[s] >= INF) continue;
            inset.clear();
            int c = 0, stored = 0;
            for (int e = s; e < len; ++e) {
                int np[2], k = 0;
                for (int p : {pa[e], pb[e]})
                    if (p >= 0 && p < rp.begin + s && std::find(inset.begin(), inset.end(), p) == inset.end() &&
                        !(k == 1 && np[0] == p))                 // the same value twice counts once
                        np[k++] = p;
                if (e > s && c + cost[e] + (int)inset.size() + k > budget) break;
                for (int q = 0; q < k; ++q) {
                    inset.push_back(np[q]);
                    stored += !S.again[np[q] - rp.begin];
                }
                c += cost[e];
                const int end = e + 1;
                const int64_t w = (s == 0 || end == len) ? 0 : (int64_t)stored;
                const int64_t cand = best[s] + (w << 20) + 1;
                if (cand < best[end]) {
                    best[end] = cand;
                    from[end] = s;
                }
            }
        }
        std::vector<int> cuts;
        for (int e = len; e > 0; e = from[e]) cuts.push_back(e);
        S.start.insert(S.start.end(), cuts.rbegin(), cuts.rend());
    }
    S.pa = pa;
    S.pb = pb;
    const int K = (int)S.start.size() - 1;
    S.in.assign(K, {});
    S.store.assign(K, {});
    for (int j = 0; j < K; ++j) {
        auto &v = S.in[j];
        for (int i = S.start[j]; i < S.start[j + 1]; ++i)
            for (int p : {pa[i], pb[i]})
                if (p >= 0 && p < rp.begin + S.start[j]) v.push_back(p);
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        if (j >= 1 && j + 1 < K)
            for (int p : v)
                if (!S.again[p - rp.begin] && !S.slot.count(p)) {
                    S.slot[p] = S.ck_count++;
                    S.store[j].push_back(p);
                }
    }
    return S;
}

// The value pass with its local partials and the reverse sweep of one root
// (checkpointed when the plan has several segments): returns the NIE value,
// G[0..n) receives the interval gradient.  Returns the checkpoint intervals
// per lane the function uses.
int write_adjoint(std::string &out, const Compiled &P, int r, const std::string &name, int budget, int gl,
                  int64_t *units) {
    Decls decl;
    std::vector<std::string> body;
    PassWriter w(P, r, 0, 0, false, true, gl);
    const SegPlan S = plan_segments(P, r, budget);
    std::string ret;
    if (S.start.size() <= 2) {
        std::vector<std::string> tan;
        w.emit(decl, body, ret, tan);
        body.push_back(w.zero_gradient());
        w.reverse(decl, body);
    } else {
        w.adjoint(decl, body, S);
        ret = "nie";
    }
    out += "__device__ __forceinline__ Iv " + name + "(const SpecLane &L, bool go, uint32_t &bad, Iv (&G)[" +
           std::to_string(P.n_vars) + "]) {\n";
    out += "    // " + std::to_string(S.start.size() - 1) + " segment(s), " + std::to_string(S.ck_count) +
           " checkpoint intervals\n";
    body.push_back(w.gradient_out());
    for (const auto &d : decl.v) out += "    " + d + "\n";
    write_guarded(out, body);
    out += "    return " + ret + ";\n}\n";
    // instruction-passes: value pass and sweep, plus the recomputation of every segment but the last
    const int len = P.roots[r].len, K = (int)S.start.size() - 1;
    *units += 2 * (int64_t)len + (K > 1 ? S.start[K - 1] : 0);
    return S.ck_count;
}

// A pass over one root's cone as a function: C == 0 returns the value; C > 0
// also writes G[0..C).  Returns which components of the root's gradient are
// structurally zero.
std::vector<bool> write_pass(std::string &out, const Compiled &P, int r, int C, int c0, bool point,
                             const std::string &name) {
    Decls decl;
    std::vector<std::string> body, tan;
    std::string val;
    PassWriter(P, r, C, c0, point).emit(decl, body, val, tan);
    out += "__device__ __forceinline__ Iv " + name + "(const SpecLane &L, bool go, uint32_t &bad";
    if (C > 0) out += ", Iv (&G)[" + std::to_string(C) + "]";
    out += ") {\n";
    for (const auto &d : decl.v) out += "    " + d + "\n";
    write_guarded(out, body);
    std::vector<bool> zero(C);
    for (int t = 0; t < C; ++t) {
        out += "    G[" + std::to_string(t) + "] = " + tan[t] + ";\n";
        zero[t] = is_zero(tan[t]);
    }
    out += "    return " + val + ";\n}\n";
    return zero;
}

// Whether some node lies in more than one root's cone: the union program is
// then shorter than the root programs together.
bool roots_share_nodes(const Compiled &P) {
    int64_t sum = 0;
    for (const auto &rp : P.roots) sum += rp.len;
    return P.uprog.len < sum;
}

// A pass over the union of the root cones (PassWriter::emit_union): the point
// pass fills FC, the value pass V, a tangent pass adds its components' terms of
// every root's mean value form to acc (and the first sets nie, the values).
void write_union_pass(std::string &out, const Compiled &P, int C, int c0, bool point, const std::string &name) {
    Decls decl;
    std::vector<std::string> body;
    PassWriter(P, (int)P.roots.size(), C, c0, point).emit_union(decl, body);
    out += "__device__ __forceinline__ void " + name + "(const SpecLane &L, bool go, uint32_t &bad, ";
    out += C > 0 ? "Iv (&acc)[N_ROOTS], Iv (&nie)[N_ROOTS]" : point ? "Iv (&FC)[N_ROOTS]" : "Iv (&V)[N_ROOTS]";
    out += ") {\n";
    for (const auto &d : decl.v) out += "    " + d + "\n";
    write_guarded(out, body);
    out += "}\n";
}

// Peak number of intervals a tangent pass over components cmask keeps live:
// every value from its instruction to its last read, each with its
// structurally nonzero components in the pass.
int peak_live(const Compiled &P, const RootProg &rp, uint64_t cmask) {
    const int len = rp.len;
    std::vector<uint64_t> dep(len);                       // variables the value of instruction pc depends on
    std::vector<int> last(len, -1), prod(std::max(rp.n_slots, 1) + 1, -1);
    auto operand = [&](uint32_t kind, uint32_t a, int pc) -> uint64_t {
        if (kind == K_VAR) return a < 64 ? 1ull << a : 0;
        if (kind != K_SLOT || a >= prod.size() || prod[a] < 0) return 0;
        last[prod[a]] = pc;
        return dep[prod[a]];
    };
    for (int pc = 0; pc < len; ++pc) {
        const Dec I = decode(P.instr[rp.begin + pc]);
        uint64_t m = operand(I.ak, I.a, pc);
        if (I.op <= I_DIV) m |= operand(I.bk, I.b, pc);
        dep[pc] = m;
        if (I.d >= prod.size()) prod.resize(I.d + 1, -1);
        prod[I.d] = pc;
    }
    // a root's value lives to the end of its own program; in the union pass
    // each root is consumed where it is computed
    if (&rp != &P.uprog && rp.result_slot >= 0 && (size_t)rp.result_slot < prod.size() && prod[rp.result_slot] >= 0)
        last[prod[rp.result_slot]] = len;
    std::vector<int> delta(len + 2, 0);                   // live intervals: + at the definition, - after the last read
    for (int pc = 0; pc < len; ++pc) {
        const int w = 1 + __builtin_popcountll(dep[pc] & cmask);
        delta[pc] += w;
        delta[std::max(last[pc], pc) + 1] -= w;
    }
    int cur = 0, peak = 0;
    for (int pc = 0; pc < len; ++pc) peak = std::max(peak, cur += delta[pc]);
    return peak;
}

// Default tangent chunk: the fewest passes whose live intervals stay near the
// register file (values recomputed per pass cost more than a few spills, a
// register file overflowing into scratch costs more than an extra pass).
constexpr int LIVE_LIMIT = 100;     // intervals (4 VGPRs each)

int default_chunk(const Compiled &P) {
    const int n = P.n_vars;
    for (int passes = 1; passes <= n; ++passes) {
        const int c = (n + passes - 1) / passes;
        if (passes > 1 && c == (n + passes - 2) / (passes - 1)) continue;   // same chunk as one pass fewer
        int peak = 0;
        for (int c0 = 0; c0 < n; c0 += c) {
            const int cw = std::min(c, n - c0);
            const uint64_t cmask = (cw >= 64 ? ~0ull : ((1ull << cw) - 1)) << c0;
            peak = std::max(peak, peak_live(P, P.uprog, cmask));
        }
        if (peak <= LIVE_LIMIT) return c;
    }
    return 1;
}

}  // namespace

int spec_plan(const Compiled &P, const mvf_spec_options *opt, int *chunk, int64_t *units) {
    const int n = P.n_vars;
    const int grad = opt ? opt->grad : MVF_GRAD_FWD;
    if (grad < MVF_GRAD_FWD || grad > MVF_GRAD_AUTO) return set_error(MVF_EINVAL, "bad grad");
    const bool fwd = grad != MVF_GRAD_REV, rev = grad != MVF_GRAD_FWD;
    int c = opt && opt->chunk > 0 ? opt->chunk : 0;
    if (c == 0) c = fwd ? default_chunk(P) : 1;
    if (c < 1 || c > n) return set_error(MVF_EINVAL, "chunk out of range [1, n]");
    if (opt && opt->ckpt_budget > MAX_CKPT_BUDGET)
        return set_error(MVF_EINVAL, "ckpt_budget above " + std::to_string(MAX_CKPT_BUDGET) + " intervals");
    if (rev && opt && opt->waves == 1)
        return set_error(MVF_EINVAL, "the adjoint kernels are not built for one wave per SIMD");
    const int passes = (n + c - 1) / c;
    // value pass, and the centre and tangent passes of the forward mode, over
    // the union of the root cones when roots share nodes, else per root; per
    // root the adjoint's centre pass, value pass, recomputation and sweep (at
    // most four passes over its program)
    int64_t sum = 0;
    for (const auto &rp : P.roots) sum += rp.len;
    const bool share = roots_share_nodes(P);
    int64_t u = share ? (int64_t)P.uprog.len * (1 + (fwd ? 1 + passes : 0)) : sum * (1 + (fwd ? passes : 0));
    if (!share || rev) u += sum;
    if (rev) u += 3 * sum;
    const int64_t cap = opt && opt->max_code > 0 ? opt->max_code : DEFAULT_MAX_CODE;
    *chunk = c;
    *units = u;
    if (u > cap)
        return set_error(MVF_ELIMIT, "tape too large to specialise: " + std::to_string(u) + " instruction-passes > " +
                                         std::to_string(cap));
    return MVF_OK;
}

int spec_ckpt_budget(const Compiled &P, const mvf_spec_options *opt, int waves) {
    if (opt && opt->ckpt_budget != 0) return opt->ckpt_budget;
    // the register file in intervals (four VGPRs each) less working
    // registers, at most MAX_CKPT_BUDGET.  Larger segments spill more but
    // store fewer checkpoints, and checkpoint traffic is what bounds the
    // segmented adjoint: on the 32-variable workload budget 32 ran 16 % faster
    // than 12 (which the register file less the gradient would give); on the
    // 8-variable batch workload 32 ran faster than 20, 24 and 28.  With more
    // than 16 variables part of the gradient stays in VGPRs (spec_gl_count):
    // there 24 is taken, which on the 32-variable workload ran 3 % faster than
    // 32 with the whole gradient in VGPRs and 4 % faster with 16 components in
    // LDS (20 within 1 % of 24, 28 2-5 % slower).
    const int regs = 128 / std::max(1, waves);
    const int b = std::min(MAX_CKPT_BUDGET, std::max(12, regs - 8));
    return P.n_vars > 16 ? std::min(b, 24) : b;
}

int spec_ckpt_min_records(const Compiled &P, const mvf_spec_options *opt, int waves) {
    // The library's choice segments every root of a tape whose largest root
    // keeps more partials in its single-pass adjoint than twice the register
    // file holds (measured: mid, 114 partials, is faster in one pass; the batch
    // workload, 239, faster with every root segmented), and none otherwise; an
    // explicit budget segments every root.
    if (opt && opt->ckpt_budget != 0) return 0;
    return P.max_rec > 2 * 128 / std::max(1, waves) ? 0 : INT32_MAX;
}

void spec_ckpt_plan_stats(const Compiled &P, int32_t *segments, int32_t *stored, int32_t *loaded) {
    const int waves = 2;
    const int budget = spec_ckpt_budget(P, nullptr, waves), min_records = spec_ckpt_min_records(P, nullptr, waves);
    *segments = *stored = *loaded = 0;
    for (int r = 0; r < (int)P.roots.size(); ++r) {
        const SegPlan S = plan_segments(P, r, P.roots[r].n_rec > min_records ? budget : -1);
        const int K = (int)S.start.size() - 1;
        *segments += K;
        *stored += S.ck_count;
        for (int j = 1; j + 1 < K; ++j)
            for (int p : S.in[j]) *loaded += !S.again[p - P.roots[r].begin];
    }
}

std::string spec_source(const Compiled &P, int chunk, int waves, int grad, int ckpt_budget, int min_records,
                        int *ck_count, int64_t *units) {
    const int n = P.n_vars, m = (int)P.roots.size();
    const bool fwd = grad != MVF_GRAD_REV, rev = grad != MVF_GRAD_FWD;
    std::string s;
    s += "// generated: specialised bounding kernels, " + std::to_string(n) + " variables, " + std::to_string(m) +
         " roots" + (fwd ? ", tangent mode with " + std::to_string(chunk) + " components per pass" : "") +
         (rev ? ", reverse-mode adjoint" : "") + "\n";
    s += "#define MVF_SPEC_WAVES " + std::to_string(waves) + "\n";
    if (fwd) s += "#define MVF_SPEC_FWD 1\n";
    if (rev) s += "#define MVF_SPEC_REV 1\n";
    s += "#include \"mvf_spec.h\"\nnamespace mvf {\nnamespace dev {\nnamespace spec {\n";
    s += "constexpr int N_VARS = " + std::to_string(n) + ", N_ROOTS = " + std::to_string(m) +
         ", N_GL = " + std::to_string(rev ? spec_gl_count(P, waves) : 0) + ";\n";
    s += "template <bool REV>\n__device__ uint32_t lane(const SpecLane &L, int mode, bool go, const LaneOut &o, "
         "FeasTrack &F);\n";
    int ck = 0;
    int64_t u = 0;                      // instruction-passes generated
    // Roots whose cones share nodes are computed by passes over the union of
    // the cones (each shared node once per pass); disjoint cones by a pass per
    // root (the same work, and each root's partial state stays out of the
    // other roots' passes: measured 2 % faster on the batch workload's forward
    // kernels).  The adjoints, each with its root's centre pass, are per root.
    const bool share = roots_share_nodes(P);
    std::vector<std::vector<bool>> zero(m, std::vector<bool>(n));     // structurally zero gradient components
    if (share) {
        u += (int64_t)P.uprog.len * (1 + (fwd ? 1 + (n + chunk - 1) / chunk : 0));
        if (fwd) write_union_pass(s, P, 0, 0, true, "upoint");
        write_union_pass(s, P, 0, 0, false, "uvalue");
        if (fwd)
            for (int c0 = 0; c0 < n; c0 += chunk)
                write_union_pass(s, P, std::min(chunk, n - c0), c0, false, "utangent_" + std::to_string(c0));
    }
    for (int r = 0; r < m; ++r) {
        const std::string R = std::to_string(r);
        const int64_t len = P.roots[r].len;
        if (!share || rev) {
            write_pass(s, P, r, 0, 0, true, "point_" + R);
            u += len;
        }
        if (!share) {
            u += len * (1 + (fwd ? (n + chunk - 1) / chunk : 0));
            write_pass(s, P, r, 0, 0, false, "value_" + R);
            if (fwd)
                for (int c0 = 0; c0 < n; c0 += chunk) {
                    const auto z = write_pass(s, P, r, std::min(chunk, n - c0), c0, false,
                                              "tangent_" + R + "_" + std::to_string(c0));
                    for (size_t t = 0; t < z.size(); ++t) zero[r][c0 + t] = z[t];
                }
        }
        if (rev)
            ck = std::max(ck, write_adjoint(s, P, r, "adjoint_" + R, P.roots[r].n_rec > min_records ? ckpt_budget : -1,
                                            spec_gl_count(P, waves), &u));
    }
    // The bound of every root: the value over the box (NIE), or the mean value
    // form from the centre value and the gradient (intersected with the value
    // unless the mode is MVF alone); then the checks, the reduction and the
    // branch-and-bound tracking root by root, as the interpreter's bound_lane.
    auto finish = [&](std::string &t, const std::string &ind, const std::string &R, const std::string &B,
                      const std::string &FC) {
        t += ind + "if (" + B + ".lo != " + B + ".lo || " + B + ".nh != " + B + ".nh) bad = 1;\n";
        t += ind + "reduce_root(" + R + ", N_ROOTS, " + B + ", o);\n";
        t += ind + "track_root(F, " + R + ", " + B + ", " + FC + ", mode != MVF_MODE_NIE, o);\n";
    };
    auto mvf_of = [](const std::string &acc, const std::string &nie) {
        return "mode == MVF_MODE_MVF ? " + acc + " : Iv{fmax_(" + acc + ".lo, " + nie + ".lo), fmax_(" + acc +
               ".nh, " + nie + ".nh)}";
    };
    // NIE mode with shared nodes: one value pass over the union for every root
    auto nie_union = [&](std::string &t) {
        t += "    if (mode == MVF_MODE_NIE) {\n        Iv B[N_ROOTS];\n        uvalue(L, go, bad, B);\n";
        for (int r = 0; r < m; ++r) finish(t, "        ", std::to_string(r), "B[" + std::to_string(r) + "]", "kZero");
        t += "        return bad;\n    }\n";
    };
    // one root's block: its bound from the lines in mvf (which set FC and B), or
    // in NIE mode from its value pass (roots with disjoint cones)
    auto root_block = [&](std::string &t, const std::string &R, const std::string &mvf) {
        t += "    {\n        Iv B, FC = kZero;\n";
        if (share) {
            t += mvf;
        } else {
            t += "        if (mode == MVF_MODE_NIE) {\n            B = value_" + R + "(L, go, bad);\n        } else {\n";
            std::string ind;
            for (size_t a = 0, b; a < mvf.size(); a = b + 1) {
                b = mvf.find('\n', a);
                ind += "    " + mvf.substr(a, b - a + 1);
            }
            t += ind + "        }\n";
        }
        finish(t, "        ", R, "B", "FC");
        t += "    }\n";
    };
    if (rev) {
        // the reverse-mode adjoint of each root in turn, its centre value next
        // to it (a centre pass over the union ahead of all adjoints would keep
        // every root's value live across them)
        s += "template <>\n__device__ __forceinline__ uint32_t lane<true>(const SpecLane &L, int mode, bool go, "
             "const LaneOut &o, FeasTrack &F) {\n    uint32_t bad = 0;\n";
        if (share) nie_union(s);
        for (int r = 0; r < m; ++r) {
            const std::string R = std::to_string(r);
            std::string b = "        FC = point_" + R + "(L, go, bad);\n";
            b += "        Iv G[N_VARS];\n        const Iv nie = adjoint_" + R + "(L, go, bad, G);\n";
            b += "        Iv acc = FC;\n";
            for (int i = 0; i < n; ++i)
                b += "        const Iv d" + std::to_string(i) + " = spec_dx(L, " + std::to_string(i) + ");\n";
            for (int i = 0; i < n; ++i)
                b += "        acc = iadd(acc, imul_dx(G[" + std::to_string(i) + "], d" + std::to_string(i) + "));\n";
            b += "        B = " + mvf_of("acc", "nie") + ";\n";
            root_block(s, R, b);
        }
        s += "    return bad;\n}\n";
    }
    if (ck_count) *ck_count = ck;
    if (units) *units = u;
    const std::string n_pf = "constexpr int N_CK = " + std::to_string(rev ? ck : 0) + ";\n";
    if (!fwd) {
        s += n_pf + "}  // namespace spec\n}  // namespace dev\n}  // namespace mvf\n#include \"mvf_spec_kernel.h\"\n";
        return s;
    }
    s += "template <>\n__device__ __forceinline__ uint32_t lane<false>(const SpecLane &L, int mode, bool go, "
         "const LaneOut &o, FeasTrack &F) {\n    uint32_t bad = 0;\n";
    if (share) {
        // the tangent passes over the union, each adding its components' terms
        nie_union(s);
        s += "    Iv FCs[N_ROOTS], acc[N_ROOTS], nie[N_ROOTS];\n    upoint(L, go, bad, FCs);\n";
        for (int r = 0; r < m; ++r) s += "    acc[" + std::to_string(r) + "] = FCs[" + std::to_string(r) + "];\n";
        for (int c0 = 0; c0 < n; c0 += chunk) s += "    utangent_" + std::to_string(c0) + "(L, go, bad, acc, nie);\n";
        for (int r = 0; r < m; ++r) {
            const std::string R = std::to_string(r);
            root_block(s, R, "        FC = FCs[" + R + "];\n        B = " + mvf_of("acc[" + R + "]", "nie[" + R + "]") + ";\n");
        }
    } else {
        // every root in turn: its centre pass, then its tangent passes
        for (int r = 0; r < m; ++r) {
            const std::string R = std::to_string(r);
            std::string b = "        FC = point_" + R + "(L, go, bad);\n        Iv acc = FC, nie = kZero;\n";
            for (int c0 = 0; c0 < n; c0 += chunk) {
                const int c = std::min(chunk, n - c0);
                b += "        {\n            Iv G[" + std::to_string(c) + "];\n";
                b += "            const Iv v = tangent_" + R + "_" + std::to_string(c0) + "(L, go, bad, G);\n";
                if (c0 == 0) b += "            nie = v;\n";
                // the factors X_i - c_i first (their LDS reads issued together), then the
                // products; a zero component adds nothing
                for (int t = 0; t < c; ++t)
                    if (!zero[r][c0 + t])
                        b += "            const Iv d" + std::to_string(t) + " = spec_dx(L, " + std::to_string(c0 + t) +
                             ");\n";
                for (int t = 0; t < c; ++t)
                    if (!zero[r][c0 + t])
                        b += "            acc = iadd(acc, imul_dx(G[" + std::to_string(t) + "], d" + std::to_string(t) +
                             "));\n";
                b += "        }\n";
            }
            b += "        B = " + mvf_of("acc", "nie") + ";\n";
            root_block(s, R, b);
        }
    }
    s += "    return bad;\n}\n";
    s += n_pf + "}  // namespace spec\n}  // namespace dev\n}  // namespace mvf\n";
    s += "#include \"mvf_spec_kernel.h\"\n";
    return s;
}

namespace {

uint64_t fnv1a(const std::string &s, uint64_t h = 1469598103934665603ull) {
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

// $MVF_SPEC_CACHE, else _spec_cache/ beside the library itself (so a tree
// that carries the library carries its compiled kernels too)
std::string cache_dir() {
    const char *e = std::getenv("MVF_SPEC_CACHE");
    if (e && *e) return std::string(e) == "off" ? "" : std::string(e);
    Dl_info di;
    if (dladdr(reinterpret_cast<void *>(&cache_dir), &di) && di.dli_fname) {
        std::string lib = di.dli_fname;
        const size_t slash = lib.rfind('/');
        return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/_spec_cache";
    }
    const char *home = std::getenv("HOME");
    return home && *home ? std::string(home) + "/.cache/mvf_spec" : "";
}

void mkdirs(const std::string &d) {
    for (size_t p = 1; p <= d.size(); ++p)
        if (p == d.size() || d[p] == '/') mkdir(d.substr(0, p).c_str(), 0755);
}

bool read_file(const std::string &path, std::vector<char> &out) {
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) return false;
    std::fseek(f, 0, SEEK_END);
    const long sz = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    out.resize(sz > 0 ? (size_t)sz : 0);
    const bool ok = sz > 0 && std::fread(out.data(), 1, out.size(), f) == out.size();
    std::fclose(f);
    return ok;
}

void write_file_atomic(const std::string &path, const std::vector<char> &data) {
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    const bool ok = std::fwrite(data.data(), 1, data.size(), f) == data.size();
    std::fclose(f);
    if (ok) std::rename(tmp.c_str(), path.c_str());
    else std::remove(tmp.c_str());
}

}  // namespace

int spec_compile(const std::string &src, const std::string &arch, bool use_cache, std::vector<char> &code,
                 bool *from_cache, double *seconds) {
    const auto t0 = std::chrono::steady_clock::now();
    *from_cache = false;
    std::vector<std::string> opts = {"--offload-arch=" + arch, "-O3", "-std=c++17", "-ffp-contract=off",
                                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    int ver_major = 0, ver_minor = 0;
    hiprtcVersion(&ver_major, &ver_minor);
    std::string key = src;
    for (const auto &o : opts) key += "\n" + o;
    for (size_t i = 0; i < k_spec_header_count; ++i) key += k_spec_header_src[i];
    key += "\nhiprtc " + std::to_string(ver_major) + "." + std::to_string(ver_minor);
    char hex[17];
    std::snprintf(hex, sizeof hex, "%016" PRIx64, fnv1a(key));
    if (const char *dump = std::getenv("MVF_SPEC_DUMP")) {       // a copy of the generated source, for inspection
        FILE *f = std::fopen(dump, "w");
        if (f) {
            std::fwrite(src.data(), 1, src.size(), f);
            std::fclose(f);
        }
    }
    const std::string dir = use_cache ? cache_dir() : "";
    const std::string path = dir.empty() ? "" : dir + "/mvf_spec_" + hex + ".co";
    if (!path.empty() && read_file(path, code)) {
        utime(path.c_str(), nullptr);                // last use, for pruning stale entries
        *from_cache = true;
        *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return MVF_OK;
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "mvf_spec.hip", (int)k_spec_header_count, k_spec_header_src,
                            k_spec_header_name) != HIPRTC_SUCCESS)
        return set_error(MVF_EHIP, "hiprtcCreateProgram failed");
    std::vector<const char *> po;
    for (const auto &o : opts) po.push_back(o.c_str());
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)po.size(), po.data());
    if (rc != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls, '\0');
        if (ls) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        if (log.size() > 4000) log = log.substr(0, 4000) + "...";
        return set_error(MVF_EHIP, std::string("hiprtc: ") + hiprtcGetErrorString(rc) + "\n" + log);
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    code.resize(cs);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    if (!path.empty()) {
        mkdirs(dir);
        write_file_atomic(path, code);
    }
    *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return MVF_OK;
}

size_t spec_lds_bytes(int tab_total, int m, int gl) {
    size_t b = (size_t)tab_total * 32;
    b += ((size_t)(BLK / 64) * (2 * m + 5) * 8 + 15) & ~(size_t)15;
    b += (2 * MVF_MAX_VARS + 8) * 4;
    if (gl > 0) b = ((b + 15) & ~(size_t)15) + (size_t)gl * BLK * 16;
    return b;
}

int spec_gl_count(const Compiled &P, int waves) {
    // Tapes whose adjoint the library segments (section on MAX_CKPT_BUDGET)
    // keep up to 16 gradient components in LDS beside the tables (16 x 256
    // lanes x 16 bytes = 64 KB per workgroup, two workgroups per CU at two
    // waves per SIMD), the last ones of a larger gradient.  On the 8-variable
    // batch workload the whole gradient in LDS freed the 32 VGPRs that the
    // kernels spilled (no scratch left): 38.5 ms steadily against 39.6-49 ms;
    // the 10-variable workload ran the same; on the 32-variable workload 16
    // components in LDS halved the scratch per lane and ran 4 % faster (8 or
    // 12 had changed nothing there); the 6-variable mid tape, kept in one pass,
    // ran 4 % slower.  A table too large to sit beside them makes mvf_bound's
    // automatic choice take the interpreter.
    const bool segmented = spec_ckpt_min_records(P, nullptr, waves) == 0;
    return waves <= 2 && segmented ? std::min(P.n_vars, 16) : 0;
}

}  // namespace mvf
