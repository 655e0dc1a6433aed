"""Readers for the paper-value fixtures under tests/golden/ (entries as printed)."""
import ast
import math
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def num(expr: str) -> float:
    """Evaluate a printed closed form made of numbers, + - * / and sqrt()."""
    tree = ast.parse(expr.strip(), mode="eval")

    def ev(n):
        if isinstance(n, ast.Expression):
            return ev(n.body)
        if isinstance(n, ast.Constant) and isinstance(n.value, (int, float)):
            return float(n.value)
        if isinstance(n, ast.UnaryOp) and isinstance(n.op, (ast.USub, ast.UAdd)):
            v = ev(n.operand)
            return -v if isinstance(n.op, ast.USub) else v
        if isinstance(n, ast.BinOp) and isinstance(n.op, (ast.Add, ast.Sub, ast.Mult, ast.Div)):
            a, b = ev(n.left), ev(n.right)
            return {ast.Add: a + b, ast.Sub: a - b, ast.Mult: a * b, ast.Div: a / b}[type(n.op)]
        if isinstance(n, ast.Call) and isinstance(n.func, ast.Name) and n.func.id == "sqrt" and len(n.args) == 1:
            return math.sqrt(ev(n.args[0]))
        raise ValueError(f"unsupported expression {expr!r}")

    return ev(tree)


def lines(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        for ln in fh:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                yield ln


def time_R():
    out, cur = {}, None
    for ln in lines("time_R.txt"):
        if ln.startswith("order"):
            cur = int(ln.split()[1]); out[cur] = []
        else:
            out[cur].append([num(x) for x in ln.split(";")])
    return out


def prism_basis():
    sec, nodes, monos, basis = None, [], [], {}
    for ln in lines("prism_basis.txt"):
        if ln in ("nodes", "monomials"):
            sec = ln; continue
        if ln.startswith("basis"):
            sec = int(ln.split()[1]); basis[sec] = {}; continue
        if sec == "nodes":
            nodes.append([num(x) for x in ln.split(";")])
        elif sec == "monomials":
            monos = [tuple(int(v) for v in t.split()) for t in ln.split(";")]
        else:
            for item in ln.split(";"):
                e, v = item.split("=")
                basis[sec][tuple(int(t) for t in e.split())] = num(v)
    return nodes, monos, basis


def square_rules():
    out, cur = {}, None
    for ln in lines("square_quadrature.txt"):
        if ln.startswith("rule"):
            cur = ln.split()[1]; out[cur] = []
        else:
            out[cur].append([num(x) for x in ln.split(";")])
    return out


def prism_order2_update():
    """rows of D_xi, D_eta, D_zeta at the six second-order nodes"""
    out = []
    for ln in lines("prism_order2_update.txt"):
        out.append([[num(x) for x in part.split(";")] for part in ln.split("|")])
    return out


def prism_order4_nodes():
    sec, nodes, monos = None, [], []
    for ln in lines("prism_order4_nodes.txt"):
        if ln in ("nodes", "monomials"):
            sec = ln; continue
        if sec == "nodes":
            nodes.append([num(x) for x in ln.split(";")])
        else:
            monos = [tuple(int(v) for v in t.split()) for t in ln.split(";")]
    return nodes, monos


def icosahedral_angles():
    return [(int(a), num(b), int(c)) for a, b, c in (ln.split(";") for ln in lines("icosahedral_angles.txt"))]


def triangle_rules():
    out, cur = {}, None
    for ln in lines("triangle_quadrature.txt"):
        if ln.startswith("rule"):
            cur = ln.split()[1]; out[cur] = []
        else:
            out[cur].append([num(x) for x in ln.split(";")])
    return out
