"""CPU checks of the C ABI: the library loads, exports every entry point that
include/lb.h declares, the ctypes structs match the C layout, and the default
options are the paper's Section 4 values. No GPU work is done here."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lb.h")
LIB = os.path.join(ROOT, "paper_2603_03933_amd", "liblbtr.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="liblbtr.so not built (run __graft_entry__.build())")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for n in ("lb_energy_grad", "lb_hessvec", "lb_tr_subproblem", "lb_imex_tr_solve", "lb_plan_create", "lb_plan_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2603_03933_amd import lb

    L = lb.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) == set(lb.exported_symbols())


def test_struct_layouts_match_c():
    from paper_2603_03933_amd import lb

    structs = {
        "lb_grid": lb.LbGrid,
        "lb_params": lb.LbParams,
        "lb_sub_opts": lb.LbSubOpts,
        "lb_sub_info": lb.LbSubInfo,
        "lb_tr_opts": lb.LbTrOpts,
        "lb_tr_info": lb.LbTrInfo,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            cf = "lambda" if fname == "lambda_" else fname
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {cf}));')
    lines.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-std=c99", "-o", exe, src], check=True)
        out = subprocess.run([exe], check=True, stdout=subprocess.PIPE, text=True).stdout
    got = {}
    for line in out.splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)



def header_prototypes():
    """{name: (return type, [parameter declarations])} of every prototype in lb.h."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"^([a-z][\w ]*?\**)\s*\b(lb_[a-z_0-9]+)\s*\(([^)]*)\)\s*;", text, flags=re.M):
        args = [a.strip() for a in " ".join(m.group(3).split()).split(",")]
        out[m.group(2)] = (m.group(1).strip(), [a for a in args if a and a != "void"])
    return out


def _c_kind(decl):
    if "*" in decl:
        return "ptr"
    words = decl.split()[:-1]  # drop the parameter name
    return {("double",): "f64", ("int",): "i32", ("long",): "i64", ("size_t",): "u64",
            ("unsigned", "long", "long"): "u64"}[tuple(words)]


def _py_kind(ct):
    if ct in (ctypes.c_void_p, ctypes.c_char_p) or issubclass(ct, ctypes._Pointer):
        return "ptr"
    return {ctypes.c_double: "f64", ctypes.c_int: "i32", ctypes.c_long: "i64", ctypes.c_size_t: "u64",
            ctypes.c_ulonglong: "u64"}[ct]


def test_binding_signatures_match_the_header():
    """Every entry point's parameter list and return type in the ctypes
    binding agree with its prototype in lb.h (count and kind of each
    argument), so no call passes a value where the library reads another."""
    from paper_2603_03933_amd import lb

    protos = header_prototypes()
    assert set(protos) == set(lb._SIGS)
    for name, (ret, args) in protos.items():
        pres, pargs = lb._SIGS[name]
        assert [_c_kind(a) for a in args] == [_py_kind(t) for t in pargs], name
        if ret == "void":
            assert pres is None, name
        elif "*" in ret:
            assert pres is ctypes.c_char_p, name
        else:
            assert _py_kind(pres) == {"int": "i32", "size_t": "u64"}[ret], name

def test_default_options_are_section4_values():
    from paper_2603_03933_amd import lb

    o = lb.tr_opts()
    assert (o.gamma_c, o.gamma_e, o.gamma_lambda, o.theta) == (0.5, 2.0, 1.5, 1e-4)
    assert (o.mu_lo, o.mu_hi, o.mu0, o.r0, o.nu0) == (1.0, 1e5, 1.0, 1.0, 5.0)
    assert o.eps == 1e-10 and o.grad_norm_inf == 1
    assert o.eta == 0.1 and o.sub.eps_sub == 1e-13
    s = lb.sub_opts()
    assert s.eta == 0.1 and s.eps_sub == 1e-13 and s.max_inner > 0


def test_version_and_error_string():
    from paper_2603_03933_amd import lb

    assert lb.lib().lb_version() >= 100
    assert isinstance(lb.lib().lb_last_error(), bytes)


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No CPU fallback: a missing library raises, and CPU tensors are rejected."""
    import torch

    from paper_2603_03933_amd import lb

    monkeypatch.setattr(lb, "_lib", None)
    monkeypatch.setattr(lb, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        lb.lib()
    with pytest.raises(TypeError):
        lb._ptr(torch.zeros(4, dtype=torch.float64), 4, "psi")


def test_plan_rejects_bad_grids_without_touching_the_gpu():
    """Argument errors are caught on the host before any device call."""
    from paper_2603_03933_amd import lb

    L = lb.lib()
    h = ctypes.c_void_p()
    g = lb.LbGrid()
    g.dim = 4
    assert L.lb_plan_create(ctypes.byref(h), ctypes.byref(g), 1, 0, None) == -1
    assert "dim" in L.lb_last_error().decode()
    g.dim = 2
    g.n[0], g.n[1] = 10, 16  # 10 = 2 * 5: no radix-5 passes
    g.box[0], g.box[1] = 1.0, 1.0
    assert L.lb_plan_create(ctypes.byref(h), ctypes.byref(g), 1, 0, None) < 0
    g.n[0] = 16
    assert L.lb_plan_create(ctypes.byref(h), ctypes.byref(g), 9, 0, None) == -1  # batch limit
    assert L.lb_plan_create(ctypes.byref(h), ctypes.byref(g), 1, 7, None) < 0  # no such precision
