// mvf_tape.cpp -- tape validation and compilation into per-root register programs.
//
// The DAG of a factorable function (Sec. 2.2 "Factorable function"; Sec. 3.2,
// Fig. DAG_NIE) is evaluated by every lane on its own subdomain.  Each root's
// cone (the nodes it depends on) becomes a straight program in node-index
// order.  Variable and constant leaves are folded into operand fields, and
// intermediate results are assigned register slots by linear-scan liveness,
// so one program serves value passes and tangent passes of any chunk size.
#include <math.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <climits>
#include <cstring>

#include "mvf_internal.h"

namespace mvf {

namespace {

bool is_leaf(int op) { return op == MVF_VAR || op == MVF_CONST; }
bool is_binary(int op) { return op >= MVF_ADD && op <= MVF_DIV; }
bool is_unary(int op) { return (op >= MVF_SQR && op <= MVF_LOG) || (op >= MVF_TANH && op <= MVF_COS); }

// instruction opcode of a tape op (the general forms; constant-operand forms are chosen later)
uint32_t instr_op(int op) {
    return op == MVF_TANH ? I_TANH : op == MVF_SIN ? I_SIN : op == MVF_COS ? I_COS : (uint32_t)op;
}

// Reference FP64 op counts (value, per tangent component, adjoint) of one
// instruction; interval products use the four-endpoint form, a constant
// operand makes + - * / cheap.
void ref_cost(int op, bool a_const, bool b_const, int *val, int *tan, int *adj) {
    bool c = a_const || b_const;
    switch (op) {
    case MVF_ADD: case MVF_SUB:
        *val = 2; *tan = c ? 0 : 2; *adj = c ? 2 : 4; return;
    case MVF_MUL:
        if (c) { *val = 2; *tan = 2; *adj = 4; } else { *val = 14; *tan = 30; *adj = 32; }
        return;
    case MVF_DIV:
        if (b_const) { *val = 2; *tan = 2; *adj = 4; } else { *val = 14; *tan = 30; *adj = 32; }
        return;
    case MVF_SQR: *val = 5; *tan = 14; *adj = 18; return;
    case MVF_SQRT: *val = 2; *tan = 14; *adj = 18; return;
    case MVF_EXP: case MVF_LOG: *val = 2; *tan = 14; *adj = 16; return;
    // tanh: two library values and the clamp, then 1 - Z^2 (7 ops) once per op
    case MVF_TANH: *val = 11; *tan = 14; *adj = 16; return;
    // sin, cos: two library values, two extremum tests (a subtraction and a
    // quotient each) and the clamp, then the derivative (the other function) once
    case MVF_SIN: case MVF_COS: *val = 28; *tan = 14; *adj = 16; return;
    default: *val = 0; *tan = 0; *adj = 0;
    }
}

// Enclosure [RD(1/k), RU(1/k)] of 1/k for k > 0: the round-to-nearest quotient
// and its neighbour on the side of the exact value.  fma is correctly rounded,
// so the sign of fma(q, k, -1) is the sign of the exact residual q*k - 1.
void recip_enclosure(double k, double *lo, double *hi) {
    const double q = 1.0 / k;
    const double r = std::fma(q, k, -1.0);
    if (r == 0.0) { *lo = q; *hi = q; }
    else if (r > 0.0) { *lo = std::nextafter(q, -INFINITY); *hi = q; }
    else { *lo = q; *hi = std::nextafter(q, INFINITY); }
}

// Tangent cost of one node summed over the components it depends on, in the
// units of ref_cost: what the forward mode does when structurally zero
// components are skipped (a sum with a zero component is the other term, a
// product with a variable's unit component the other factor).
int64_t sparse_tan_cost(const mvf_node *nodes, const mvf_node &nd, const std::vector<uint64_t> &dep) {
    const bool bin = is_binary(nd.op);
    const int ao = nodes[nd.a].op, bo = bin ? nodes[nd.b].op : -1;
    const bool konst = ao == MVF_CONST || bo == MVF_CONST;
    const uint64_t da = dep[nd.a], db = bin ? dep[nd.b] : 0;
    int64_t c = 0;
    for (uint64_t u = da | db; u; u &= u - 1) {
        const uint64_t j = u & (~u + 1);
        const bool a = (da & j) != 0, b = (db & j) != 0;
        switch (nd.op) {
        case MVF_ADD: case MVF_SUB: c += a && b ? 2 : 0; break;
        case MVF_MUL:
            c += konst ? 2 : (a && ao != MVF_VAR ? 14 : 0) + (b && bo != MVF_VAR ? 14 : 0) + (a && b ? 2 : 0);
            break;
        case MVF_DIV:
            c += bo == MVF_CONST ? 2 : (b && bo != MVF_VAR ? 14 : 0) + (a && b ? 2 : 0) + 14;
            break;
        default: c += ao == MVF_VAR ? 0 : 14;      // the derivative times the component
        }
    }
    return c;
}

int fail(std::string *err, int code, const char *fmt, long a = 0, long b = 0) {
    if (err) {
        char buf[256];
        snprintf(buf, sizeof buf, fmt, a, b);
        *err = buf;
    }
    return code;
}

}  // namespace

int compile_tape(const mvf_node *nodes, int32_t n_nodes, const double *consts, int32_t n_consts, int32_t n_vars,
                 const int32_t *roots, int32_t n_roots, Compiled *out, std::string *err) {
    if (!nodes || !roots || !out) return fail(err, MVF_EINVAL, "null tape array");
    if (n_nodes < 1 || n_nodes > MVF_MAX_NODES) return fail(err, MVF_ELIMIT, "n_nodes %ld outside [1, %ld]", n_nodes, MVF_MAX_NODES);
    if (n_vars < 1 || n_vars > MVF_MAX_VARS) return fail(err, MVF_ELIMIT, "n_vars %ld outside [1, %ld]", n_vars, MVF_MAX_VARS);
    if (n_roots < 1 || n_roots > MVF_MAX_ROOTS) return fail(err, MVF_ELIMIT, "n_roots %ld outside [1, %ld]", n_roots, MVF_MAX_ROOTS);
    if (n_consts < 0 || (n_consts > 0 && !consts)) return fail(err, MVF_EINVAL, "bad constant array");
    for (int i = 0; i < n_nodes; ++i) {
        const mvf_node &nd = nodes[i];
        if (nd.op < MVF_VAR || nd.op > MVF_COS) return fail(err, MVF_ETAPE, "node %ld: bad opcode %ld", i, nd.op);
        if (nd.op == MVF_VAR && (nd.a < 0 || nd.a >= n_vars))
            return fail(err, MVF_ETAPE, "node %ld: variable index %ld out of range", i, nd.a);
        if (nd.op == MVF_CONST) {
            if (nd.a < 0 || nd.a >= n_consts) return fail(err, MVF_ETAPE, "node %ld: constant index %ld out of range", i, nd.a);
            if (!isfinite(consts[nd.a])) return fail(err, MVF_ETAPE, "node %ld: constant %ld is not finite", i, nd.a);
        }
        if ((is_binary(nd.op) || is_unary(nd.op)) && (nd.a < 0 || nd.a >= i))
            return fail(err, MVF_ETAPE, "node %ld: operand a=%ld is not an earlier node", i, nd.a);
        if (is_binary(nd.op) && (nd.b < 0 || nd.b >= i))
            return fail(err, MVF_ETAPE, "node %ld: operand b=%ld is not an earlier node", i, nd.b);
    }
    for (int r = 0; r < n_roots; ++r)
        if (roots[r] < 0 || roots[r] >= n_nodes) return fail(err, MVF_ETAPE, "root %ld = %ld is not a node", r, roots[r]);

    Compiled C;
    C.n_vars = n_vars;
    std::vector<uint8_t> in_cone(n_nodes), in_regs(n_nodes);
    std::vector<int32_t> slot_of(n_nodes, -1), last_use(n_nodes, -1), uses(n_nodes, 0);
    std::vector<double> aux;            // reciprocal enclosures of constant divisors, (lo, -hi) pairs
    int64_t sum_val = 0, sum_tan = 0, sum_adj = 0, n_ops = 0, sum_tan_sparse = 0, combine_sparse = 0;
    // variables each node depends on: its structurally nonzero tangent components
    std::vector<uint64_t> dep(n_nodes, 0);
    for (int i = 0; i < n_nodes; ++i) {
        const mvf_node &nd = nodes[i];
        if (nd.op == MVF_VAR) dep[i] = nd.a < 64 ? 1ull << nd.a : 0;
        else if (is_binary(nd.op)) dep[i] = dep[nd.a] | dep[nd.b];
        else if (is_unary(nd.op)) dep[i] = dep[nd.a];
    }
    for (int r = 0; r < n_roots; ++r) combine_sparse += 16 * __builtin_popcountll(dep[roots[r]]) + 2;

    // Programs 0 .. m-1 compute one root each (bounding, gradients of one root);
    // program m is the union of all root cones with every root kept live to
    // its end (point values of all roots and their vector-Jacobian product).
    std::vector<uint8_t> is_root(n_nodes);
    for (int pi = 0; pi <= n_roots; ++pi) {
        const bool uni = pi == n_roots;
        RootProg P;
        P.begin = (int32_t)C.instr.size();
        std::fill(in_cone.begin(), in_cone.end(), 0);
        std::fill(is_root.begin(), is_root.end(), 0);
        int top = 0;
        for (int r = uni ? 0 : pi; r < (uni ? n_roots : pi + 1); ++r) {
            in_cone[roots[r]] = 1;
            is_root[roots[r]] = 1;
            top = std::max(top, (int)roots[r]);
        }
        for (int i = top; i >= 0; --i) {
            if (!in_cone[i]) continue;
            if (is_binary(nodes[i].op) || is_unary(nodes[i].op)) in_cone[nodes[i].a] = 1;
            if (is_binary(nodes[i].op)) in_cone[nodes[i].b] = 1;
        }
        if (!uni && is_leaf(nodes[roots[pi]].op)) {
            const mvf_node &rn = nodes[roots[pi]];
            uint32_t ak = rn.op == MVF_VAR ? K_VAR : K_CONST;
            double k = rn.op == MVF_CONST ? consts[rn.a] : 0.0;
            C.instr.push_back(make_instr(I_LOAD, ak, rn.op == MVF_VAR ? (uint32_t)rn.a : 0, K_SLOT, 0, 0, k));
            P.len = 1; P.result_slot = 0; P.n_slots = 1;
            C.roots.push_back(P);
            continue;
        }
        // program order of the arithmetic nodes, their uses and last uses
        std::vector<int32_t> order;
        for (int i = 0; i <= top; ++i)
            if (in_cone[i] && !is_leaf(nodes[i].op)) order.push_back(i);
        for (int i : order) { last_use[i] = -1; uses[i] = 0; in_regs[i] = 0; }
        for (size_t p = 0; p < order.size(); ++p) {
            const mvf_node &nd = nodes[order[p]];
            if (!is_leaf(nodes[nd.a].op)) { last_use[nd.a] = (int32_t)p; ++uses[nd.a]; }
            if (is_binary(nd.op) && !is_leaf(nodes[nd.b].op)) { last_use[nd.b] = (int32_t)p; ++uses[nd.b]; }
        }
        for (int i : order)
            if (is_root[i]) last_use[i] = INT32_MAX;        // roots stay live to the end of the program
        auto refs = [&](int j, int i) {          // operand references of node j to node i
            const mvf_node &nd = nodes[j];
            return (nd.a == i ? 1 : 0) + (is_binary(nd.op) && nd.b == i ? 1 : 0);
        };
        // linear scan over a pool of slots (lowest free id first); slot 0 is reserved
        // for results consumed only by the next instruction
        std::vector<uint8_t> busy(1, 1);
        auto take = [&]() {
            for (size_t s = 0; s < busy.size(); ++s)
                if (!busy[s]) { busy[s] = 1; return (int32_t)s; }
            busy.push_back(1);
            return (int32_t)busy.size() - 1;
        };
        auto operand = [&](int node, uint32_t *kind, uint32_t *idx, double *k) {
            const mvf_node &nd = nodes[node];
            if (nd.op == MVF_VAR) { *kind = K_VAR; *idx = (uint32_t)nd.a; }
            else if (nd.op == MVF_CONST) { *kind = K_CONST; *idx = 0; *k = consts[nd.a]; }
            else if (in_regs[node]) { *kind = K_SLOT; *idx = 0; }
            else { *kind = K_SLOT; *idx = (uint32_t)slot_of[node]; }
        };
        for (size_t p = 0; p < order.size(); ++p) {
            const int i = order[p];
            const mvf_node &nd = nodes[i];
            const bool bin = is_binary(nd.op);
            const bool a_const = nodes[nd.a].op == MVF_CONST, b_const = bin && nodes[nd.b].op == MVF_CONST;
            uint32_t ak, a, bk = K_SLOT, b = 0, init = 0;
            double ka = 0.0, kb = 0.0;
            if (a_const && b_const) {
                // materialise operand a: a load whose only consumer is this instruction
                C.instr.push_back(make_instr(I_LOAD, K_CONST, 0, K_SLOT, 0, 0, consts[nodes[nd.a].a]));
                C.instr.back().w0 |= W0_NOWRITE;
                ak = K_SLOT; a = 0;
                init |= 1u;
            } else {
                operand(nd.a, &ak, &a, &ka);
            }
            if (bin) operand(nd.b, &bk, &b, &kb);
            // release operands dying here; a dying operand's adjoint receives its first
            // contribution here in the reverse sweep (written instead of accumulated)
            if (!is_leaf(nodes[nd.a].op) && last_use[nd.a] == (int32_t)p) {
                if (!in_regs[nd.a]) busy[slot_of[nd.a]] = 0;
                init |= 1u;
            }
            if (bin && !is_leaf(nodes[nd.b].op) && last_use[nd.b] == (int32_t)p) {
                if (!in_regs[nd.b] && nd.b != nd.a) busy[slot_of[nd.b]] = 0;
                if (nd.b != nd.a) init |= 2u;
            }
            // the result stays in registers when the next node is its only consumer
            const bool nowrite = !is_root[i] && p + 1 < order.size() && uses[i] == refs(order[p + 1], i) &&
                                 uses[i] > 0;
            int32_t d = 0;
            if (nowrite) in_regs[i] = 1;
            else { d = take(); slot_of[i] = d; }

            // constant-operand forms: the other operand moves to position a
            uint32_t op = instr_op(nd.op);
            double k = a_const && !b_const ? ka : kb;
            const bool one_const = bin && (a_const != b_const);
            if (one_const) {
                const uint32_t xk = a_const ? bk : ak, xi = a_const ? b : a;
                const uint32_t xinit = a_const ? (init >> 1) & 1u : init & 1u;
                bool special = true;
                switch (nd.op) {
                case MVF_ADD: op = I_ADDK; break;
                case MVF_SUB: op = a_const ? I_KSUB : I_ADDK; if (!a_const) k = -k; break;
                case MVF_MUL:
                    if (k == 0.0) special = false;
                    else { op = std::signbit(k) ? I_MULKN : I_MULK; k = std::fabs(k); }
                    break;
                case MVF_DIV:
                    if (a_const || k == 0.0) { special = false; break; }
                    op = std::signbit(k) ? I_DIVKN : I_DIVK;
                    k = std::fabs(k);
                    b = (uint32_t)(aux.size() / 2);       // aux record index, relocated below
                    {
                        double lo, hi;
                        recip_enclosure(k, &lo, &hi);
                        aux.push_back(lo);
                        aux.push_back(-hi);
                    }
                    break;
                default: special = false;
                }
                if (special) {
                    if (op != I_DIVK && op != I_DIVKN) b = 0;
                    ak = xk; a = xi; bk = K_CONST;
                    init = xinit;
                }
            }
            Instr ins = make_instr(op, ak, a, bk, b, (uint32_t)d, k);
            ins.w0 |= (init & 1u ? W0_INIT_A : 0u) | (init & 2u ? W0_INIT_B : 0u) | (nowrite ? W0_NOWRITE : 0u);
            C.instr.push_back(ins);
            P.n_rec += n_records(op, ak, bk);
            // Algorithmic work: values, tangents and the centre pass once per
            // node of the union of the root cones (a node shared by several
            // roots is computed once); an adjoint sweep per root over its cone.
            int cv, ct, ca;
            ref_cost(nd.op, a_const, b_const, &cv, &ct, &ca);
            if (uni) {
                sum_val += cv; sum_tan += ct; ++n_ops;
                sum_tan_sparse += sparse_tan_cost(nodes, nd, dep);
                if (nd.op == MVF_SQR || nd.op == MVF_SQRT) sum_val += 2;   // 2U or 1/(2Z), once per op
            } else {
                sum_adj += ca;
            }
        }
        if (!uni) {
            P.len = (int32_t)C.instr.size() - P.begin;
            P.result_slot = slot_of[roots[pi]];
            P.n_slots = (int32_t)busy.size();
            C.roots.push_back(P);
            continue;
        }
        // union program: variable and constant roots are loaded at its end (in the
        // reverse sweep their seeds reach the gradient before any other contribution)
        for (int r = 0; r < n_roots; ++r) {
            const mvf_node &rn = nodes[roots[r]];
            if (!is_leaf(rn.op)) { C.union_slots.push_back(slot_of[roots[r]]); continue; }
            const int32_t d = take();
            C.instr.push_back(make_instr(I_LOAD, rn.op == MVF_VAR ? K_VAR : K_CONST, rn.op == MVF_VAR ? (uint32_t)rn.a : 0,
                                         K_SLOT, 0, (uint32_t)d, rn.op == MVF_CONST ? consts[rn.a] : 0.0));
            C.union_slots.push_back(d);
        }
        P.len = (int32_t)C.instr.size() - P.begin;
        P.result_slot = -1;
        P.n_slots = (int32_t)busy.size();
        C.uprog = P;
    }
    // Layout: [root programs][auxiliary records][root records] -- what the bounding
    // kernels stage -- then [union program][union record][union root slots].
    std::vector<Instr> uni(C.instr.begin() + C.uprog.begin, C.instr.end());
    C.instr.resize(C.uprog.begin);
    C.n_prog = (int32_t)C.instr.size();
    if (C.n_prog + aux.size() / 2 > 65536)
        return fail(err, MVF_ELIMIT, "program of %ld instructions exceeds 65536 records", (long)(C.n_prog + aux.size() / 2));
    auto relocate = [&](Instr &ins) {
        const uint32_t op = ins.w0 & 31u;
        if (op == I_DIVK || op == I_DIVKN) ins.w1 = (ins.w1 & 0xffff0000u) | ((ins.w1 & 0xffffu) + (uint32_t)C.n_prog);
    };
    for (auto &ins : C.instr) relocate(ins);
    for (auto &ins : uni) relocate(ins);
    for (size_t j = 0; j < aux.size(); j += 2) {
        Instr rec;
        std::memcpy(&rec, &aux[j], 16);
        C.instr.push_back(rec);
    }
    for (auto &P : C.roots) {
        C.max_slots = std::max(C.max_slots, P.n_slots);
        C.max_rec = std::max(C.max_rec, P.n_rec);
    }
    // one record per root: program begin, length, result slot, reverse-mode record count
    C.root_base = (int32_t)C.instr.size();
    for (auto &P : C.roots) {
        const uint32_t w[4] = {(uint32_t)P.begin, (uint32_t)P.len, (uint32_t)P.result_slot, (uint32_t)P.n_rec};
        Instr rec;
        std::memcpy(&rec, w, 16);
        C.instr.push_back(rec);
    }
    C.n_bound = (int32_t)C.instr.size();
    C.uprog.begin = (int32_t)C.instr.size();
    C.instr.insert(C.instr.end(), uni.begin(), uni.end());
    // the union record {begin, length, records, roots}, then the root slots, four per record
    C.union_base = (int32_t)C.instr.size();
    {
        const uint32_t w[4] = {(uint32_t)C.uprog.begin, (uint32_t)C.uprog.len, (uint32_t)C.uprog.n_rec,
                               (uint32_t)n_roots};
        Instr rec;
        std::memcpy(&rec, w, 16);
        C.instr.push_back(rec);
        for (int r = 0; r < n_roots; r += 4) {
            uint32_t q[4] = {0, 0, 0, 0};
            for (int j = 0; j < 4 && r + j < n_roots; ++j) q[j] = (uint32_t)C.union_slots[r + j];
            std::memcpy(&rec, q, 16);
            C.instr.push_back(rec);
        }
    }
    if (C.instr.size() > 65536)
        return fail(err, MVF_ELIMIT, "program of %ld records exceeds 65536", (long)C.instr.size());

    // value passes keep every slot in registers
    const int avail = usable_dwords(n_roots);
    C.union_ok = C.uprog.n_slots * 4 <= avail;
    if (C.max_slots * 4 > avail)
        return fail(err, MVF_ELIMIT, "a root needs %ld live slots; the slot file holds %ld values", C.max_slots, avail / 4);

    const int64_t n = n_vars, m = n_roots;
    C.ref_fwd = sum_val + n * sum_tan + 2 * n_ops + m * (16 * n + 2) + 10 * n;
    C.ref_rev = sum_val + sum_adj + 2 * n_ops + m * (16 * n + 2) + 10 * n;
    C.ref_fwd_sparse = sum_val + sum_tan_sparse + 2 * n_ops + combine_sparse + 10 * n;
    *out = std::move(C);
    return MVF_OK;
}

}  // namespace mvf
