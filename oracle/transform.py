"""The CNF-to-circuit transformation (the paper's Algorithm 1, Section
"Transformation Algorithm") with its Boolean expressions as truth tables --
TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Clauses are lists of non-zero ints (DIMACS literals: +x is variable x, -x its
negation).  The algorithm appends clauses one at a time to the sub-clause
list SC; after each append it tries every variable v of SC that is neither a
primary input nor an intermediate variable as the output of SC:

* f = FindBooleanExpression(v, SC): the conjunction, over the clauses of SC
  that contain the literal -v, of the clause with -v removed (the condition
  under which v = 1 satisfies them);
* g = FindBooleanExpression(-v, SC): the same over the clauses containing +v
  with +v removed (the condition under which v = 0 satisfies them);
* v is the output of SC when f is the complement of g.  Then the expression
  is recorded; v becomes a primary output if f is constant, else an
  intermediate variable; every other variable of SC that is not an
  intermediate variable is appended to the primary inputs; SC is emptied.

Readings this oracle takes (the paper leaves them open):

* candidates are tried in decreasing variable index (this reproduces the
  orientation of the gates in the paper's Fig. 1 example);
* f and g are tables over the variables of SC other than v, ascending
  variable index = ascending digit of the row (variable slot 0 least
  significant); "Simplify" is represented by the support of f (the
  variables f depends on) -- two-level minimisation is a separate step;
* an under-specified SC (no output found and no variable of SC occurs in a
  later clause) becomes an expression with an auxiliary output constrained to
  1: the conjunction of SC over all its variables; its variables that are not
  intermediate are appended to the primary inputs, and SC is emptied; the
  same applies to a non-empty SC left after the last clause;
* appending to PI skips variables already there (the lists are sets kept in
  order of first entry); a tautological clause (x and -x together) is not
  accepted.

Truth tables are Python ints (bit r = value at row r); plain loops over rows,
so only small SC (a dozen variables) are practical here.
"""
from __future__ import annotations

from dataclasses import dataclass, field


@dataclass
class Expr:
    out: int            # the output variable, 0 for an auxiliary output
    kind: str           # "IV", "PO" (constant f) or "AUX" (constrained to 1)
    first: int          # SC = clauses[first .. last]
    last: int
    vars: list          # table variables, ascending (slot j = digit j of the row)
    table: int          # bit r = f at row r (AUX: the conjunction of SC)
    support: list = field(default_factory=list)  # variables the table depends on


def _clause_value(clause, vars_, row, drop=None):
    """Truth of the clause at a row over vars_, the literal ``drop`` removed."""
    for lit in clause:
        if lit == drop:
            continue
        x = abs(lit)
        val = (row >> vars_.index(x)) & 1
        if (lit > 0 and val) or (lit < 0 and not val):
            return True
    return False


def find_expression(lit: int, sc, vars_) -> int:
    """FindBooleanExpression: the table over vars_ of the conjunction, over
    the clauses of sc containing -lit, of the clause without -lit.  (For
    lit = v this is f: v = 1 falsifies -v; for lit = -v it is g.)"""
    table = 0
    for row in range(1 << len(vars_)):
        ok = all(_clause_value(c, vars_, row, drop=-lit) for c in sc if -lit in c)
        table |= int(ok) << row
    return table


def support(table: int, nvars: int) -> list:
    """Slots j such that some pair of rows differing only in digit j differ."""
    out = []
    for j in range(nvars):
        if any(((table >> r) & 1) != ((table >> (r ^ (1 << j))) & 1) for r in range(1 << nvars)):
            out.append(j)
    return out


def transform(clauses):
    """Algorithm 1.  Returns (PO, PI, IV, exprs): variable lists in order of
    entry (PO may hold 0 for auxiliary outputs) and the Expr records."""
    for c in clauses:
        assert c and all(l != 0 for l in c) and not any(-l in c for l in c), c
    last_use = {}
    for i, c in enumerate(clauses):
        for l in c:
            last_use[abs(l)] = i
    PO, PI, IV, exprs = [], [], [], []
    start = 0

    def sc_vars(a, b):
        return sorted({abs(l) for c in clauses[a:b + 1] for l in c})

    def add_inputs(vs, skip):
        for w in vs:
            if w not in IV and w != skip and w not in PI:
                PI.append(w)

    i = 0
    while i < len(clauses):
        sc = clauses[start:i + 1]
        vs = sc_vars(start, i)
        found = False
        for v in sorted(vs, reverse=True):
            if v in PI or v in IV:
                continue
            others = [x for x in vs if x != v]
            f = find_expression(v, sc, others)
            g = find_expression(-v, sc, others)
            full = (1 << (1 << len(others))) - 1
            if f == (~g) & full:
                const = f in (0, full)
                (PO if const else IV).append(v)
                exprs.append(Expr(v, "PO" if const else "IV", start, i, others, f,
                                  [others[j] for j in support(f, len(others))]))
                add_inputs(vs, v)
                start, found = i + 1, True
                break
        if not found and all(last_use[x] <= i for x in vs):
            # under-specified: the conjunction of SC, output constrained to 1
            t = 0
            for row in range(1 << len(vs)):
                t |= int(all(_clause_value(c, vs, row) for c in sc)) << row
            PO.append(0)
            exprs.append(Expr(0, "AUX", start, i, vs, t, [vs[j] for j in support(t, len(vs))]))
            add_inputs(vs, None)
            start = i + 1
        i += 1
    return PO, PI, IV, exprs


def parse_dimacs(text: str):
    """Clauses of a DIMACS CNF text (comment lines 'c', header 'p cnf')."""
    clauses, cur = [], []
    for line in text.splitlines():
        s = line.strip()
        if not s or s[0] in "cp%":
            continue
        for tok in s.split():
            v = int(tok)
            if v == 0:
                if cur:
                    clauses.append(cur)
                cur = []
            else:
                cur.append(v)
    if cur:
        clauses.append(cur)
    return clauses
