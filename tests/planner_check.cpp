// Host check of the evaluation planner (runtime.cpp, compiled here for the
// CPU and linked against the built library for the device-side symbols it
// names; no device call is made).  Random populations are hash-consed into
// DAGs on the host in the device's node order (first occurrence, children
// before parents), planned by the sequential and the level-parallel decision
// passes, and every emitted program is run on a host stack machine:
//   - no program underflows its stack or needs more than D slots, and each
//     leaves exactly one value;
//   - a fill program reads only cache rows of lower levels;
//   - fill programs run level by level, then every reduce and store
//     program gives, at every test case, bit for bit the value of direct
//     evaluation of its root node (operand orders of the reversed and
//     permuted opcodes included);
//   - with the same number of stack spills the two decision passes cache
//     the same nodes at the same levels;
//   - the sequential and level-parallel preparations mark the same
//     variable-free subtrees for folding and list the same operator nodes
//     by height;
//   - a cache budget too small for the spills gives TGP_ENOMEM.
#include "runtime.cpp"

#include <cstdio>
#include <map>
#include <random>
#include <tuple>

namespace {

int g_bad = 0;
#define CHECK(c, ...)                          \
    do {                                       \
        if (!(c)) {                            \
            if (g_bad < 20) printf(__VA_ARGS__); \
            ++g_bad;                           \
        }                                      \
    } while (0)

// Host operators for the subset the random trees use.  min and max order
// -0 below +0 so that they are symmetric (the emitter may swap their
// operands); nothing here depends on matching the device bit for bit, only
// on the programs and the direct evaluation using the same functions.
float h_min(float a, float b) {
    if (a != a) return b;
    if (b != b) return a;
    if (a == b) return std::signbit(a) ? a : b;
    return a < b ? a : b;
}
float h_max(float a, float b) {
    if (a != a) return b;
    if (b != b) return a;
    if (a == b) return std::signbit(a) ? b : a;
    return a > b ? a : b;
}
float apply(int op, float a, float b, float c) {
    switch (op) {
    case TGP_ADD: return a + b;
    case TGP_SUB: return a - b;
    case TGP_MULT: return a * b;
    case TGP_DIV: return b == 0.0f ? 0.0f : a / b;
    case TGP_MIN: return h_min(a, b);
    case TGP_MAX: return h_max(a, b);
    case TGP_MDIST: return a * 0.5f + b * 0.5f;
    case TGP_NEG: return -a;
    case TGP_ABS: return std::fabs(a);
    case TGP_CLIP: return h_max(h_min(a, c), b);
    case TGP_IF: return a != 0.0f ? b : c;
    default: return NAN;
    }
}

const int kOps[] = {TGP_ADD, TGP_SUB, TGP_MULT, TGP_DIV, TGP_MIN, TGP_MAX, TGP_MDIST,
                    TGP_NEG, TGP_ABS, TGP_CLIP, TGP_IF};

struct Gen {
    std::mt19937_64 rng;
    explicit Gen(uint64_t s) : rng(s) {}
    double u() { return std::uniform_real_distribution<double>(0, 1)(rng); }
    int below(int n) { return (int)(rng() % (uint64_t)n); }
};

// A random tree in postfix (op, var, value); grow or full to max depth.
struct Tok {
    int op, var;
    float value;
};
void random_tree(Gen &g, int depth, bool full, std::vector<Tok> &out) {
    const bool leaf = depth == 0 || (!full && g.u() < 0.3);
    if (leaf) {
        if (g.u() < 0.6) out.push_back({TGP_VAR, g.below(2), 0.0f});
        else out.push_back({TGP_CONST, 0, (float)(g.below(9) - 4) * 0.25f});  // few distinct constants
        return;
    }
    const int op = kOps[g.below((int)(sizeof kOps / sizeof kOps[0]))];
    for (int i = 0; i < kArity[op]; ++i) random_tree(g, depth - 1, full, out);
    out.push_back({op, 0, 0.0f});
}

// Hash-consing of postfix trees into d (structural identity).
struct Builder {
    tgp_dag_s &d;
    std::map<std::tuple<int, int, uint32_t, int, int, int>, int32_t> ids;
    explicit Builder(tgp_dag_s &dag) : d(dag) {}
    int32_t add_tree(const std::vector<Tok> &t) {
        std::vector<int32_t> st;
        for (const Tok &k : t) {
            const int a = kArity[k.op];
            int32_t c[3] = {-1, -1, -1};
            for (int j = a - 1; j >= 0; --j) {
                c[j] = st.back();
                st.pop_back();
            }
            uint32_t vb;
            memcpy(&vb, &k.value, 4);
            auto key = std::make_tuple(k.op, k.var, vb, c[0], c[1], c[2]);
            auto it = ids.find(key);
            int32_t id;
            if (it != ids.end()) {
                id = it->second;
            } else {
                id = (int32_t)d.op.size();
                ids.emplace(key, id);
                d.op.push_back(k.op | (k.var << 8));
                d.value.push_back(k.value);
                int32_t h = 0;
                for (int j = 0; j < 3; ++j) {
                    d.kid.push_back(c[j]);
                    if (c[j] >= 0) h = std::max(h, d.height[c[j]] + 1);
                }
                d.height.push_back(h);
            }
            st.push_back(id);
        }
        return st.back();
    }
};

void make_dag(tgp_dag_s &d, Gen &g, int n_ind, int n_ch, int d_max) {
    Builder b(d);
    d.n_ind = n_ind;
    d.n_ch = n_ch;
    for (int r = 0; r < n_ind * n_ch; ++r) {
        std::vector<Tok> t;
        random_tree(g, 1 + r % d_max, (r / 2) % 2 == 0, t);
        d.roots.push_back(b.add_tree(t));
    }
    d.stats.dag_nodes = (int64_t)d.op.size();
    d.stats.n_roots = (int64_t)d.roots.size();
}

// Stack-machine run of one program at one case; false on a malformed
// program (stack misuse or depth above D).
bool run(const Plan &P, const ProgDesc &pd, int D, float x, float y, const std::vector<float> &cache,
         float *out, std::vector<int32_t> *reads) {
    float s[64];
    int sp = 0;
    for (uint32_t i = 0; i < pd.len; ++i) {
        const uint2 ins = P.code_host[pd.code_off + i];
        const uint32_t c = ins.x & 0xffu;
        if ((int)(ins.x >> 8) != sp) return false;  // the depth the word carries
        if (c == I_END) {
            if (sp != 1) return false;
            *out = s[0];
            return true;
        }
        if (c <= I_CACHE) {
            if (sp >= D) return false;
            float v = 0;
            if (c == I_X) v = x;
            else if (c == I_Y) v = y;
            else if (c == I_CONST) memcpy(&v, &ins.y, 4);
            else if (c == I_CACHE) {
                v = cache[ins.y];
                if (reads) reads->push_back((int32_t)ins.y);
            } else return false;  // no z axis here
            s[sp++] = v;
            continue;
        }
        if (c >= kFuseBase) {  // fused form: the terminal operand is read here
            const uint32_t kind = (c - kFuseBase) / 16, v = (c - kFuseBase) % 16;
            if (kind > kFuseCache || v >= (uint32_t)kNumFused || sp < 1) return false;
            float t = 0;
            if (kind == kFuseX) t = x;
            else if (kind == kFuseY) t = y;
            else if (kind == kFuseConst) memcpy(&t, &ins.y, 4);
            else {
                t = cache[ins.y];
                if (reads) reads->push_back((int32_t)ins.y);
            }
            s[sp - 1] = kFuseRev[v] ? apply(kFuseOps[v], t, s[sp - 1], 0) : apply(kFuseOps[v], s[sp - 1], t, 0);
            continue;
        }
        int op, ar;
        const uint8_t *order;
        static const uint8_t ident[3] = {0, 1, 2}, rev[2] = {1, 0};
        if (c >= kPermBase) {
            const int t = (int)(c - kPermBase) / 6, p = (int)(c - kPermBase) % 6;
            op = t == 0 ? TGP_CLIP : (t == 1 ? TGP_IF : TGP_LERP);
            ar = 3;
            order = kPerms[p];
        } else if (c >= kRevBase) {
            op = (int)(c - kRevBase);
            ar = 2;
            order = rev;
        } else if (c >= kFnBase) {
            op = (int)(c - kFnBase);
            ar = kArity[op];
            order = ident;
        } else {
            return false;
        }
        if (sp < ar) return false;
        const int dst = sp - ar;
        float arg[3] = {0, 0, 0};
        for (int q = 0; q < ar; ++q) arg[order[q]] = s[dst + q];  // slot dst+q holds child order[q]
        s[dst] = apply(op, arg[0], arg[1], arg[2]);
        sp = dst + 1;
    }
    return false;  // no I_END
}

void check_plan(const char *what, tgp_dag_s &d, PlanJob &w, int D, Gen &g) {
    const Plan &P = d.plan;
    const Planner &pl = w.pl;
    const int64_t U = d.stats.dag_nodes;
    const int n_cases = 6;
    for (int cs = 0; cs < n_cases; ++cs) {
        const float x = cs == 0 ? 0.0f : (float)(g.u() * 4 - 2), y = cs == 1 ? -0.0f : (float)(g.u() * 4 - 2);
        std::vector<float> val(U);
        for (int64_t n = 0; n < U; ++n) {
            const int op = d.op[n] & 0xff;
            const int32_t *k = &d.kid[3 * n];
            if (op == TGP_VAR) val[n] = ((d.op[n] >> 8) & 0xff) == 0 ? x : y;
            else if (op == TGP_CONST) val[n] = d.value[n];
            else val[n] = apply(op, val[k[0]], k[1] >= 0 ? val[k[1]] : 0.0f, k[2] >= 0 ? val[k[2]] : 0.0f);
        }
        std::vector<float> cache(P.n_slots, NAN);
        for (size_t l = 0; l + 1 < P.level_first.size(); ++l)
            for (int32_t i = P.level_first[l]; i < P.level_first[l + 1]; ++i) {
                const ProgDesc &pd = P.fill_host[i];
                std::vector<int32_t> reads;
                float v;
                const bool ok = run(P, pd, D, x, y, cache, &v, &reads);
                CHECK(ok, "%s: fill program %d malformed\n", what, i);
                if (!ok) continue;
                const int32_t node = P.slot_node[pd.dest];
                CHECK(pl.level[node] == (int32_t)l, "%s: slot %d filled at level %zu, planned %d\n", what, pd.dest, l,
                      pl.level[node]);
                for (int32_t r : reads)
                    CHECK(pl.level[P.slot_node[r]] < (int32_t)l, "%s: level %zu reads slot %d of level %d\n", what, l, r,
                          pl.level[P.slot_node[r]]);
                CHECK(memcmp(&v, &val[node], 4) == 0, "%s: fill of node %d gives %a, direct %a\n", what, node, v,
                      val[node]);
                cache[pd.dest] = v;
            }
        for (const ProgDesc &pd : P.reduce_host) {
            float v;
            const bool ok = run(P, pd, D, x, y, cache, &v, nullptr);
            CHECK(ok, "%s: reduce program malformed\n", what);
            const int32_t node = w.reduce_list[pd.dest].first;
            CHECK(!ok || memcmp(&v, &val[node], 4) == 0, "%s: root node %d gives %a, direct %a\n", what, node, v,
                  val[node]);
        }
        for (const ProgDesc &pd : P.store_host) {
            float v;
            const bool ok = run(P, pd, D, x, y, cache, &v, nullptr);
            CHECK(ok, "%s: store program malformed\n", what);
            const int32_t node = d.roots[pd.dest];
            CHECK(!ok || memcmp(&v, &val[node], 4) == 0, "%s: stored root %d gives %a, direct %a\n", what, node, v,
                  val[node]);
        }
    }
}

}  // namespace

int main() {
    Gen g(20260514);
    struct Case {
        int n_ind, n_ch, d_max, D;
        double access;
    };
    // small and large (the large ones take the level-parallel decisions)
    const Case cases[] = {{40, 1, 6, 8, 20.0},  {40, 2, 9, 4, 20.0},   {300, 3, 10, 8, 2.0},
                          {300, 1, 12, 5, -1.0}, {2500, 3, 11, 8, 20.0}, {2500, 3, 12, 4, 20.0},
                          {2500, 1, 12, 6, 2.0}, {2500, 2, 12, 8, -1.0}};
    for (const Case &c : cases) {
        tgp_dag_s d;
        make_dag(d, g, c.n_ind, c.n_ch, c.d_max);
        const int64_t U = d.stats.dag_nodes;
        int64_t spills[2] = {0, 0};
        std::vector<uint8_t> cached[2];
        std::vector<int32_t> level[2];
        for (int threads : {1, 8}) {
            char what[160];
            snprintf(what, sizeof what, "U=%lld D=%d access=%g threads=%d", (long long)U, c.D, c.access, threads);
            d.plan = Plan();
            PlanJob w(&d, 4096, c.D, (size_t)1 << 24);
            plan_prepare(w, false);
            const tgp_status st = plan_decide_emit(w, c.D, true, c.access, 0, threads);
            CHECK(st == TGP_OK, "%s: status %d\n", what, st);
            if (st != TGP_OK) continue;
            check_plan(what, d, w, c.D, g);
            int64_t fused[4] = {0, 0, 0, 0};  // fused forms by operand kind
            for (const uint2 &ins : d.plan.code_host) {
                const uint32_t code = ins.x & 0xffu;
                if (code >= kFuseBase && code < kFuseBase + 64) ++fused[(code - kFuseBase) / 16];
            }
            printf("%s: fused forms x %lld y %lld const %lld cache %lld\n", what, (long long)fused[0],
                   (long long)fused[1], (long long)fused[2], (long long)fused[3]);
            if (c.n_ind >= 300)
                CHECK(fused[0] > 0 && fused[1] > 0 && fused[2] > 0 && fused[3] > 0,
                      "%s: a fused operand kind never emitted\n", what);
            const int t = threads == 1 ? 0 : 1;
            spills[t] = w.pl.spills;
            cached[t] = w.pl.cached;
            level[t] = w.pl.level;
            printf("%s: slots %d spills %lld levels %zu programs %d+%d instructions %lld%s\n", what, d.plan.n_slots,
                   (long long)d.plan.n_spills, d.plan.level_first.size() - 1, d.plan.n_fill, d.plan.n_reduce,
                   (long long)d.plan.instructions, U >= kParallelDecideNodes && threads > 1 ? " (level-parallel)" : "");
            // a budget below the spills the stack bound needs is refused
            if (w.pl.spills > 1) {
                d.plan = Plan();
                PlanJob small(&d, 4096, c.D, (size_t)(w.pl.spills - 1));
                plan_prepare(small, false);
                CHECK(plan_decide_emit(small, c.D, true, c.access, 0, threads) == TGP_ENOMEM,
                      "%s: budget below the spills accepted\n", what);
            }
        }
        {  // folding preparation, sequential and level-parallel
            PlanJob a(&d, 4096, c.D, (size_t)1 << 24), b(&d, 4096, c.D, (size_t)1 << 24);
            plan_prepare(a, true, 1);
            plan_prepare(b, true, 8);
            CHECK(a.pl.folded == b.pl.folded && a.fold_first == b.fold_first && a.fold_list == b.fold_list,
                  "U=%lld: folding preparation differs between 1 and 8 threads\n", (long long)U);
            int64_t n_fold = 0;
            for (uint8_t f : a.pl.folded) n_fold += f;
            printf("U=%lld: %lld folded subtrees, %zu variable-free operator nodes\n", (long long)U,
                   (long long)n_fold, a.fold_list.size());
        }
        if (spills[0] == spills[1])
            CHECK(cached[0] == cached[1] && level[0] == level[1],
                  "U=%lld D=%d: same spills, different cached nodes or levels\n", (long long)U, c.D);
    }
    if (g_bad) {
        printf("%d failures\n", g_bad);
        return 1;
    }
    printf("OK\n");
    return 0;
}
