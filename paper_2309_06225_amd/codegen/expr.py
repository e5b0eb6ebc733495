"""A small expression-DAG builder that emits straight-line HIP device code.

The pointwise 4dST/CCZ4 algebra is described once with these nodes; the same
graph is emitted as the forward right-hand side and, by reverse-mode
accumulation over the graph, as its vector-Jacobian product.  Nodes are
hash-consed (common subexpressions are shared), constants are folded, and the
emitted code is a list of ``const double`` definitions that the HIP compiler
schedules and register-allocates.
"""
from __future__ import annotations

import math


class Graph:
    def __init__(self):
        self.nodes: list[Node] = []
        self.table: dict = {}

    def _new(self, op, a=None, b=None, val=None, name=None, c=None):
        key = (op, a.idx if a is not None else None, b.idx if b is not None else None, val, name,
               c.idx if c is not None else None)
        hit = self.table.get(key)
        if hit is not None:
            return hit
        n = Node(self, op, a, b, val, name, len(self.nodes), c)
        self.nodes.append(n)
        self.table[key] = n
        return n

    # leaves
    def const(self, v: float) -> "Node":
        v = float(v)
        if v == 0.0:
            v = 0.0  # fold -0.0
        return self._new("c", val=v)

    def input(self, name: str) -> "Node":
        return self._new("in", name=name)

    def param(self, name: str) -> "Node":
        return self._new("p", name=name)

    # arithmetic with folding
    def add(self, a, b):
        a, b = self.lift(a), self.lift(b)
        if a.is_const(0.0):
            return b
        if b.is_const(0.0):
            return a
        if a.op == "c" and b.op == "c":
            return self.const(a.val + b.val)
        if b.op == "neg":
            return self.sub(a, b.a)
        if a.op == "neg":
            return self.sub(b, a.a)
        if a.idx > b.idx:
            a, b = b, a
        return self._new("+", a, b)

    def sub(self, a, b):
        a, b = self.lift(a), self.lift(b)
        if b.is_const(0.0):
            return a
        if a.is_const(0.0):
            return self.neg(b)
        if a is b:
            return self.const(0.0)
        if a.op == "c" and b.op == "c":
            return self.const(a.val - b.val)
        if b.op == "neg":
            return self.add(a, b.a)
        return self._new("-", a, b)

    def mul(self, a, b):
        a, b = self.lift(a), self.lift(b)
        if a.is_const(0.0) or b.is_const(0.0):
            return self.const(0.0)
        if a.is_const(1.0):
            return b
        if b.is_const(1.0):
            return a
        if a.is_const(-1.0):
            return self.neg(b)
        if b.is_const(-1.0):
            return self.neg(a)
        if a.op == "c" and b.op == "c":
            return self.const(a.val * b.val)
        if a.op == "neg" and b.op == "neg":
            return self.mul(a.a, b.a)
        if a.op == "neg":
            return self.neg(self.mul(a.a, b))
        if b.op == "neg":
            return self.neg(self.mul(a, b.a))
        if a.idx > b.idx:
            a, b = b, a
        return self._new("*", a, b)

    def div(self, a, b):
        a, b = self.lift(a), self.lift(b)
        if b.is_const(1.0):
            return a
        if a.is_const(0.0):
            return self.const(0.0)
        if b.op == "c":
            return self.mul(a, 1.0 / b.val)
        if a.op == "c" and a.val == 1.0:
            return self._new("rcp", b)
        return self.mul(a, self._new("rcp", b))

    def neg(self, a):
        a = self.lift(a)
        if a.op == "c":
            return self.const(-a.val)
        if a.op == "neg":
            return a.a
        return self._new("neg", a)

    def exp(self, a):
        a = self.lift(a)
        if a.op == "c":
            return self.const(math.exp(a.val))
        return self._new("exp", a)

    def sqrt(self, a):
        """Square root (diagnostics only: the reverse mode does not handle it)."""
        return self._new("sqrt", self.lift(a))

    def fabs(self, a):
        """Absolute value (diagnostics only: the reverse mode does not handle it)."""
        a = self.lift(a)
        if a.op == "c":
            return self.const(abs(a.val))
        if a.op == "neg":
            a = a.a
        return self._new("abs", a)

    def gtabs(self, a, b):
        """Condition |a| > |b| (a boolean: only `sel` reads it)."""
        a, b = self.lift(a), self.lift(b)
        if a.op == "c" and b.op == "c":
            return self.const(1.0 if abs(a.val) > abs(b.val) else 0.0)
        if a.is_const(0.0):
            return self.const(0.0)
        return self._new("gt", a, b)

    def sel(self, cond, x, y):
        """x where cond holds, else y (cond: a `gtabs` node or a constant)."""
        x, y = self.lift(x), self.lift(y)
        if cond.op == "c":
            return x if cond.val != 0.0 else y
        if x is y:
            return x
        return self._new("sel", x, y, c=cond)

    def lift(self, x):
        if isinstance(x, Node):
            return x
        return self.const(x)

    def sum(self, terms):
        acc = self.const(0.0)
        for t in terms:
            acc = self.add(acc, t)
        return acc


class Node:
    __slots__ = ("g", "op", "a", "b", "val", "name", "idx", "c")

    def __init__(self, g, op, a, b, val, name, idx, c=None):
        self.g, self.op, self.a, self.b, self.val, self.name, self.idx = g, op, a, b, val, name, idx
        self.c = c  # third operand: the condition of a select

    def kids(self):
        return [k for k in (self.a, self.b, self.c) if k is not None]

    def is_const(self, v):
        return self.op == "c" and self.val == v

    def __add__(self, o):
        return self.g.add(self, o)

    def __radd__(self, o):
        return self.g.add(o, self)

    def __sub__(self, o):
        return self.g.sub(self, o)

    def __rsub__(self, o):
        return self.g.sub(o, self)

    def __mul__(self, o):
        return self.g.mul(self, o)

    def __rmul__(self, o):
        return self.g.mul(o, self)

    def __truediv__(self, o):
        return self.g.div(self, o)

    def __rtruediv__(self, o):
        return self.g.div(o, self)

    def __neg__(self):
        return self.g.neg(self)

    def __repr__(self):
        return f"Node({self.op},{self.idx})"


def reachable(outputs):
    """Indices of nodes needed to compute `outputs`."""
    seen = set()
    stack = [o for o in outputs]
    while stack:
        n = stack.pop()
        if n.idx in seen:
            continue
        seen.add(n.idx)
        stack.extend(n.kids())
    return seen


def vjp(g: Graph, outputs, cotangents, wrt):
    """Reverse-mode accumulation: returns nodes for sum_k cot_k d out_k / d w."""
    need = reachable(outputs)
    wrt_idx = {w.idx for w in wrt}
    # nodes that depend on any w (only they receive adjoints)
    varied = set()
    for n in g.nodes:
        if n.idx not in need:
            continue
        if n.idx in wrt_idx or any(k.idx in varied for k in n.kids()):
            varied.add(n.idx)
    adj: dict[int, Node] = {}

    def acc(x, v):
        if x.idx not in varied:
            return
        adj[x.idx] = v if x.idx not in adj else g.add(adj[x.idx], v)

    for o, c in zip(outputs, cotangents):
        acc(o, c)
    order = sorted((g.nodes[i] for i in varied), key=lambda n: -n.idx)
    for n in order:
        a = adj.get(n.idx)
        if a is None or n.op in ("in", "p", "c"):
            continue
        if n.op == "+":
            acc(n.a, a)
            acc(n.b, a)
        elif n.op == "-":
            acc(n.a, a)
            acc(n.b, g.neg(a))
        elif n.op == "*":
            acc(n.a, g.mul(a, n.b))
            acc(n.b, g.mul(a, n.a))
        elif n.op == "neg":
            acc(n.a, g.neg(a))
        elif n.op == "rcp":  # d(1/x) = -1/x^2
            acc(n.a, g.neg(g.mul(a, g.mul(n, n))))
        elif n.op == "exp":  # d exp(x) = exp(x)
            acc(n.a, g.mul(a, n))
        elif n.op == "sel":  # the adjoint goes to the operand taken
            acc(n.a, g.sel(n.c, a, 0.0))
            acc(n.b, g.sel(n.c, 0.0, a))
        elif n.op == "gt":  # piecewise constant
            continue
        else:
            raise ValueError(n.op)
    return [adj.get(w.idx, g.const(0.0)) for w in wrt]


def _lit(v: float) -> str:
    if v == 0.0:
        return "0.0"
    if math.isfinite(v) and float(repr(v)) == v and len(repr(v)) < 18:
        r = repr(v)
        return r if ("." in r or "e" in r) else r + ".0"
    return v.hex()


def count_flops(g: Graph, outputs):
    """Count of add, sub, mul, reciprocal, square-root and exponential nodes
    (1 flop each); negation, absolute value, comparisons and selects are free."""
    need = reachable(outputs)
    c = {"+": 0, "-": 0, "*": 0, "rcp": 0, "neg": 0}
    for i in need:
        op = g.nodes[i].op
        if op in c or op in ("sqrt", "abs", "exp"):
            c[op] = c.get(op, 0) + 1
    total = c["+"] + c["-"] + c["*"] + c["rcp"] + c.get("sqrt", 0) + c.get("exp", 0)
    return total, c


def register_need(outputs):
    """Sethi-Ullman register need of every node on the tree expansion of the
    graph: a leaf needs 1, a binary node max(n1, n2 + 1) with n1 >= n2."""
    need = {}
    for o in outputs:
        stack = [o]
        while stack:
            x = stack[-1]
            if x.idx in need:
                stack.pop()
                continue
            chs = x.kids()
            pend = [c for c in chs if c.idx not in need]
            if pend:
                stack.extend(pend)
                continue
            stack.pop()
            if x.op in ("c", "p"):
                need[x.idx] = 0
            elif not chs:
                need[x.idx] = 1
            else:
                v = sorted((need[c.idx] for c in chs), reverse=True)
                need[x.idx] = max(v[0], 1) if len(v) == 1 else max(v[0], v[1] + 1)
    return need


def dfs_order(outputs, heavy_first=False):
    """Post-order depth-first node order: each output's dependencies are placed
    just before it, so intermediates are computed close to their uses.  With
    heavy_first, the operand with the larger register need is visited first
    (fewer values held while the other operand is computed)."""
    need = register_need(outputs) if heavy_first else None
    order, seen = [], set()
    for o in outputs:
        stack = [(o, False)]
        while stack:
            n, done = stack.pop()
            if n.idx in seen:
                continue
            if done:
                seen.add(n.idx)
                order.append(n.idx)
                continue
            stack.append((n, True))
            chs = [ch for ch in n.kids() if ch.idx not in seen]
            if heavy_first:
                chs.sort(key=lambda c: need.get(c.idx, 0), reverse=True)
            for ch in reversed(chs):
                stack.append((ch, False))
    return order


def greedy_order(outputs, prio_order):
    """Top-down list schedule that keeps few values live: among the nodes whose
    operands are all computed, take one that frees the most operands (its last
    remaining user) net of the value it creates (an output is stored at once,
    so it stays live only for its other users); ties go to the earlier node of
    prio_order.  Constants and parameters cost nothing and come first."""
    import heapq
    prio = {i: k for k, i in enumerate(prio_order)}
    nodes = {}
    stack = list(outputs)
    while stack:
        x = stack.pop()
        if x.idx in nodes:
            continue
        nodes[x.idx] = x
        for c in x.kids():
            if c.idx not in nodes:
                stack.append(c)
    ops_of = {i: {c.idx for c in x.kids()} for i, x in nodes.items()}
    users = {i: [] for i in nodes}
    for i in nodes:
        for c in ops_of[i]:
            users[c].append(i)
    remaining = {i: len(users[i]) for i in nodes}   # users not yet scheduled
    free = {i for i, x in nodes.items() if x.op in ("c", "p")}
    order = [i for i in nodes if i in free]
    done = set(order)
    pending = {i: len(ops_of[i] - done) for i in nodes if i not in done}   # operands not yet computed

    def delta(i):
        kills = sum(1 for c in ops_of[i] if c not in free and remaining[c] == 1)
        return (1 if users[i] else 0) - kills

    heap = [(delta(i), prio.get(i, 0), i) for i, k in pending.items() if k == 0]
    heapq.heapify(heap)
    # a lazy heap: an entry whose delta has dropped since it was pushed is re-keyed
    while heap:
        d, _, i = heapq.heappop(heap)
        if i in done:
            continue
        cur = delta(i)
        if cur != d:
            heapq.heappush(heap, (cur, prio.get(i, 0), i))
            continue
        done.add(i)
        order.append(i)
        for c in ops_of[i]:
            remaining[c] -= 1
            if remaining[c] == 1 and c not in free:
                for u in users[c]:
                    if u not in done and pending.get(u) == 0:
                        heapq.heappush(heap, (delta(u), prio.get(u, 0), u))
        for u in users[i]:
            pending[u] -= 1
            if pending[u] == 0:
                heapq.heappush(heap, (delta(u), prio.get(u, 0), u))
    return order


def fusion_plan(g: Graph, seq, outputs):
    """Multiply-adds to emit as explicit fused multiply-adds.  Every add or
    subtract with a product operand takes that product into an fma (the first
    operand when both are products); a product is still computed on its own
    only where something other than such an fma uses it.  Returns
    ({add node: (product node, operand position)}, {products not emitted}).
    Fusing by this fixed rule (with compiler contraction off) makes the
    rounding of the generated code the same in every kernel that includes it."""
    plan = {}
    other_use = set()
    outs = {o.idx for o in outputs}
    for i in seq:
        n = g.nodes[i]
        k_fused = None
        if n.op in ("+", "-"):
            for k, ch in enumerate((n.a, n.b)):
                if ch.op == "*":
                    k_fused = k
                    plan[i] = (ch.idx, k)
                    break
        for k, ch in enumerate((n.a, n.b, n.c)):
            if ch is not None and k != k_fused:
                other_use.add(ch.idx)
    skipped = {m for m, _ in plan.values() if m not in other_use and m not in outs}
    return plan, skipped


def _node_expr(g, n, name_of, plan):
    """C expression of an arithmetic node (with fma fusion per plan)."""
    if n.idx in plan:
        m_idx, k = plan[n.idx]
        m = g.nodes[m_idx]
        x, y = name_of(m.a), name_of(m.b)
        other = name_of(n.b if k == 0 else n.a)
        if n.op == "+":
            return f"fma({x}, {y}, {other})"
        if k == 0:  # x*y - other
            return f"fma({x}, {y}, -{other})"
        return f"fma(-{x}, {y}, {other})"  # other - x*y
    if n.op == "+":
        return f"{name_of(n.a)} + {name_of(n.b)}"
    if n.op == "-":
        return f"{name_of(n.a)} - {name_of(n.b)}"
    if n.op == "*":
        return f"{name_of(n.a)} * {name_of(n.b)}"
    if n.op == "neg":
        return f"-{name_of(n.a)}"
    if n.op == "rcp":
        return f"1.0 / {name_of(n.a)}"
    if n.op == "sqrt":
        return f"sqrt({name_of(n.a)})"
    if n.op == "exp":
        return f"exp({name_of(n.a)})"
    if n.op == "abs":
        return f"fabs({name_of(n.a)})"
    if n.op == "gt":
        return f"fabs({name_of(n.a)}) > fabs({name_of(n.b)})"
    if n.op == "sel":
        return f"{name_of(n.c)} ? {name_of(n.a)} : {name_of(n.b)}"
    raise ValueError(n.op)


def _ctype(n) -> str:
    return "bool" if n.op == "gt" else "double"


def emit(g: Graph, outputs, out_names, input_expr, param_expr, indent="  ", prefix="t", order="dfs"):
    """Straight-line C for `outputs`.  input_expr(name) / param_expr(name)
    return C expressions for leaves; out_names are C statement templates taking
    the value expression (e.g. 'OUT(3, {})').  With order='dfs' each output
    statement is placed right after the last node it needs."""
    if order == "dfs":
        seq = dfs_order(outputs)
    elif order == "dfs_heavy":
        seq = dfs_order(outputs, heavy_first=True)
    elif order == "greedy":
        seq = greedy_order(outputs, dfs_order(outputs, heavy_first=True))
    else:
        seq = sorted(reachable(outputs))
    pos = {i: k for k, i in enumerate(seq)}
    # output statements go right after their value is computed
    after = {}
    for o, tmpl in zip(outputs, out_names):
        after.setdefault(pos[o.idx] if o.op != "c" else -1, []).append((o, tmpl))
    lines = []
    names = {}
    plan, fused = fusion_plan(g, seq, outputs)

    def name_of(n):
        return names[n.idx]

    for o, tmpl in after.get(-1, []):
        lines.append(indent + tmpl.format(_lit(o.val) if o.val >= 0 else f"({_lit(o.val)})") + ";")
    for k, i in enumerate(seq):
        n = g.nodes[i]
        if n.op == "c":
            names[i] = _lit(n.val) if n.val >= 0 else f"({_lit(n.val)})"
        elif i in fused:
            pass  # emitted inside the fma of its single user
        else:
            if n.op == "in":
                expr = input_expr(n.name)
            elif n.op == "p":
                expr = param_expr(n.name)
            else:
                expr = _node_expr(g, n, name_of, plan)
            nm = f"{prefix}{i}"
            names[i] = nm
            lines.append(f"{indent}const {_ctype(n)} {nm} = {expr};")
        for o, tmpl in after.get(k, []):
            lines.append(indent + tmpl.format(names[o.idx]) + ";")
    return "\n".join(lines)


def emit_staged(g: Graph, outputs, out_stmts, input_key, param_expr, slots, indent="  ", prefix="t", order="dfs"):
    """Straight-line C like `emit`, with every memory input staged through two
    alternating buffers of `slots` slots each (the including kernel copies them
    asynchronously from memory into fast local storage).

    The node order is the depth-first one of `emit`.  It is cut into phases of
    at most `slots` staged items each; phase j reads buffer j % 2 while the
    items of phase j + 1 are being fetched into the other buffer.
      input_key(name)  -> staging key of a graph input, e.g. ("D", 17)
      out_stmts[k]     -> (template, extra_keys): the statement of output k,
                          with '{v}' for the value and '{sN}' for the slot of
                          extra_keys[N] (items the statement itself reads).
    Emitted macros: GRF_PHASE_SYNC(); GRF_STAGE_<KIND>(buf, slot, index);
    GRF_LDS(buf, slot) for a staged value.  Returns (code, number of phases,
    largest slot count used)."""
    if order == "greedy":
        seq = greedy_order(outputs, dfs_order(outputs, heavy_first=True))
    else:
        seq = dfs_order(outputs, heavy_first=(order == "dfs_heavy"))
    pos = {i: k for k, i in enumerate(seq)}
    after = {}
    for o, st in zip(outputs, out_stmts):
        if o.op == "c":
            raise ValueError("constant output in staged emission")
        after.setdefault(pos[o.idx], []).append((o, st))
    # statement list: ("node", idx) or ("out", node, template, keys)
    stmts = []
    for k, i in enumerate(seq):
        stmts.append(("node", i))
        for o, (tmpl, keys) in after.get(k, []):
            stmts.append(("out", o, tmpl, keys))

    def keys_of(st):
        if st[0] == "node":
            n = g.nodes[st[1]]
            return [input_key(n.name)] if n.op == "in" else []
        return list(st[3])

    # phases: greedy cut, each item staged in the phase of the statement using it
    phases = [[]]       # per phase: list of statement indices
    phase_items = [{}]  # per phase: key -> slot
    for si, st in enumerate(stmts):
        ks = [k for k in keys_of(st) if k not in phase_items[-1]]
        if len(phase_items[-1]) + len(ks) > slots and phases[-1]:
            phases.append([])
            phase_items.append({})
            ks = keys_of(st)
        for k in ks:
            if k not in phase_items[-1]:
                phase_items[-1][k] = len(phase_items[-1])
        if len(phase_items[-1]) > slots:
            raise ValueError("a single statement needs more slots than available")
        phases[-1].append(si)

    lines = []
    names = {}
    plan, fused = fusion_plan(g, seq, outputs)

    def name_of(n):
        return names[n.idx]

    def stage_lines(j):
        buf = j % 2
        return [f"{indent}GRF_STAGE_{kind}({buf}, {slot}, {idx});"
                for (kind, idx), slot in sorted(phase_items[j].items(), key=lambda kv: kv[1])]

    lines += stage_lines(0)
    for j, plist in enumerate(phases):
        buf = j % 2
        lines.append(f"{indent}GRF_PHASE_SYNC();")
        if j + 1 < len(phases):
            lines += stage_lines(j + 1)
        items = phase_items[j]
        for si in plist:
            st = stmts[si]
            if st[0] == "node":
                i = st[1]
                n = g.nodes[i]
                if n.op == "c":
                    names[i] = _lit(n.val) if n.val >= 0 else f"({_lit(n.val)})"
                    continue
                if i in fused:
                    continue  # emitted inside the fma of its single user
                if n.op == "in":
                    expr = f"GRF_LDS({buf}, {items[input_key(n.name)]})"
                elif n.op == "p":
                    expr = param_expr(n.name)
                else:
                    expr = _node_expr(g, n, name_of, plan)
                nm = f"{prefix}{i}"
                names[i] = nm
                lines.append(f"{indent}const {_ctype(n)} {nm} = {expr};")
            else:
                _, o, tmpl, keys = st
                fmt = {"v": names[o.idx], "b": str(buf)}
                for q, k in enumerate(keys):
                    fmt[f"s{q}"] = str(items[k])
                lines.append(indent + tmpl.format(**fmt) + ";")
    return "\n".join(lines), len(phases), max(len(p) for p in phase_items)
