"""Static check of the benchmark and entry scripts: every name a function
reads is bound in that function, an enclosing function, the module or the
builtins.  The bench's sections only run on a GPU, so a name left behind by a
refactor would otherwise surface only there."""
import ast
import builtins
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bound_in(node) -> set:
    """Names bound directly in a function body (parameters, assignments,
    loop and with targets, imports, nested definitions, comprehension and
    exception variables), not descending into nested functions."""
    names = set()
    if isinstance(node, (ast.FunctionDef, ast.AsyncFunctionDef, ast.Lambda)):
        a = node.args
        for arg in a.posonlyargs + a.args + a.kwonlyargs:
            names.add(arg.arg)
        if a.vararg:
            names.add(a.vararg.arg)
        if a.kwarg:
            names.add(a.kwarg.arg)
    body = node.body if isinstance(node.body, list) else [node.body]
    stack = list(body)
    while stack:
        n = stack.pop()
        if isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef, ast.ClassDef)):
            names.add(n.name)
            continue
        if isinstance(n, ast.Lambda):
            continue
        if isinstance(n, ast.Name) and isinstance(n.ctx, (ast.Store, ast.Del)):
            names.add(n.id)
        elif isinstance(n, (ast.Import, ast.ImportFrom)):
            for al in n.names:
                names.add((al.asname or al.name).split(".")[0])
        elif isinstance(n, ast.ExceptHandler) and n.name:
            names.add(n.name)
        elif isinstance(n, (ast.Global, ast.Nonlocal)):
            names.update(n.names)
        stack.extend(ast.iter_child_nodes(n))
    return names


def _loads(node):
    """Names read in a function body, not descending into nested functions."""
    body = node.body if isinstance(node.body, list) else [node.body]
    stack = list(body)
    while stack:
        n = stack.pop()
        if isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef, ast.Lambda, ast.ClassDef)):
            if isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef)):
                stack.extend(n.decorator_list + n.args.defaults + n.args.kw_defaults)
            continue
        if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load):
            yield n
        stack.extend(c for c in ast.iter_child_nodes(n) if c is not None)


def _undefined(path: str):
    tree = ast.parse(open(path).read(), path)
    module = _bound_in(ast.Module(body=tree.body, type_ignores=[])) | set(dir(builtins)) | {"__file__", "__name__"}
    missing = []

    def visit(fn, scopes):
        bound = _bound_in(fn)
        for name in _loads(fn):
            if name.id not in bound and not any(name.id in s for s in scopes) and name.id not in module:
                missing.append(f"{os.path.basename(path)}:{name.lineno} {name.id}")
        for n in ast.walk(fn):
            if n is not fn and isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef, ast.Lambda)):
                # visit each nested function once, from its nearest enclosing function
                parent_fns = [p for p in ast.walk(fn) if p is not n and n in list(ast.walk(p))
                              and isinstance(p, (ast.FunctionDef, ast.AsyncFunctionDef, ast.Lambda))]
                if parent_fns and parent_fns[-1] is fn or (not parent_fns):
                    visit(n, scopes + [bound])

    for top in tree.body:
        if isinstance(top, (ast.FunctionDef, ast.AsyncFunctionDef)):
            visit(top, [])
    return sorted(set(missing))


@pytest.mark.parametrize("script", ["bench.py", "__graft_entry__.py"])
def test_no_undefined_names(script):
    assert _undefined(os.path.join(ROOT, script)) == []


def test_checker_finds_a_missing_name(tmp_path):
    p = tmp_path / "probe.py"
    p.write_text("def outer():\n    k = 1\n    def inner():\n        return k + j\n    return inner\n")
    assert _undefined(str(p)) == ["probe.py:4 j"]
