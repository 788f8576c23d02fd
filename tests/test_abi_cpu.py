"""The C-ABI library on the CPU: it loads, exports every symbol the header
declares, validates parameters before touching the GPU, and enumerates
clusters by the same rule as the oracle (implemented separately)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1901_01047_amd import build, dcax
from oracle import geometry

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(dcax.LIB_PATH):
        build.build()
    return dcax.load()


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "dcax.h")).read()
    declared = sorted(set(re.findall(r"^(?:dcax_status|const char\*)\s+(dcax_\w+)\(", hdr, re.M)))
    assert declared, "no declarations parsed"
    assert sorted(dcax.EXPORTS) == declared
    for name in declared:
        assert hasattr(lib, name)


def test_struct_layouts_match_header(tmp_path):
    """sizeof/offsetof of every ABI struct field, from gcc, equal the binding's."""
    structs = {"dcax_vertex": dcax.Vertex, "dcax_proposal": dcax.Proposal, "dcax_params": dcax.Params,
               "dcax_stats": dcax.Stats, "dcax_allocator": dcax.Allocator, "dcax_dca_params": dcax.DcaParams,
               "dcax_dca_report": dcax.DcaReport}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dcax.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)
    assert dcax.PROPOSAL_DTYPE.itemsize == ctypes.sizeof(dcax.Proposal)
    assert dcax.VERTEX_DTYPE.itemsize == ctypes.sizeof(dcax.Vertex)
    for f, _ in dcax.Proposal._fields_:
        assert dcax.PROPOSAL_DTYPE.fields[f][1] == getattr(dcax.Proposal, f).offset


@pytest.mark.parametrize("field,value", [("abi_version", 7), ("beta", -1.0), ("U", -0.5), ("K_exp", 0.0),
                                         ("n_tau", 1), ("precision", 5), ("submatrix_k", 0),
                                         ("submatrix_k", 65), ("max_order", 0), ("n_freq", -1),
                                         ("refresh_every", -3), ("warmup_sweeps", -1), ("sweep_length", -2),
                                         ("flip_share", -0.1), ("flip_share", 1.0), ("flip_share", float("nan")),
                                         ("touched_twice", 2), ("touched_twice", -1), ("reserved2", 1),
                                         ("drift_tol", -1.0), ("drift_tol", float("inf"))])
def test_create_rejects_bad_params(lib, field, value):
    p = dcax.make_params()
    setattr(p, field, value)
    h = ctypes.c_void_p()
    st = lib.dcax_walker_create(ctypes.byref(p), 1, None, None, ctypes.byref(h))
    assert st == -1 and not h.value
    assert len(lib.dcax_last_error()) > 0


def test_create_rejects_bad_propagator_tables(lib):
    """Caller-supplied G0 tables: n_spin_tables outside 0..2, tables missing
    or given without a count, and a nonzero reserved word are argument
    errors, answered before any device work."""
    h = ctypes.c_void_p()
    tab = np.zeros((1, 4, 1000))
    for mutate in (lambda p: setattr(p, "n_spin_tables", 3),
                   lambda p: setattr(p, "n_spin_tables", 1),                      # no table
                   lambda p: setattr(p, "g0_tau", tab.ctypes.data),              # table, count 0
                   lambda p: setattr(p, "reserved", 1)):
        p = dcax.make_params()
        mutate(p)
        assert lib.dcax_walker_create(ctypes.byref(p), 1, None, None, ctypes.byref(h)) == -1 and not h.value
    with pytest.raises(ValueError):
        dcax.make_params(g0_tau=np.zeros((3, 4, 1000)))
    with pytest.raises(ValueError):
        dcax.make_params(g0_Kw=np.zeros((4, 64), complex))
    p = dcax.make_params(g0_tau=np.zeros((2, 4, 1000)), g0_Kw=np.zeros((2, 4, 64), complex))
    assert p.n_spin_tables == 2 and p.g0_tau and p.g0_Kw


def test_create_rejects_degenerate_cluster_and_batch(lib):
    p = dcax.make_params(cluster=(2, 2, 1, 1))
    h = ctypes.c_void_p()
    assert lib.dcax_walker_create(ctypes.byref(p), 1, None, None, ctypes.byref(h)) == -1
    p = dcax.make_params()
    assert lib.dcax_walker_create(ctypes.byref(p), 0, None, None, ctypes.byref(h)) == -1
    two = (dcax.Params * 2)(dcax.make_params(), dcax.make_params(precision=dcax.DCAX_FP32_MIXED))
    assert lib.dcax_walker_create(two, 2, None, None, ctypes.byref(h)) == -1    # mixed precisions
    assert lib.dcax_walker_create(ctypes.byref(p), 1, None, None, None) == -1


@pytest.mark.parametrize("c", [(2, 0, 0, 2), (4, 0, 0, 4), (2, 2, 2, -2), (6, 0, 0, 6), (8, 0, 0, 8),
                               (3, 1, -1, 3)])
def test_cluster_enumeration_matches_oracle(c):
    p = dcax.make_params(cluster=c)
    sites, K = dcax.cluster(p)
    a1, a2 = (c[0], c[1]), (c[2], c[3])
    assert np.array_equal(sites, geometry.cluster_sites(a1, a2))
    assert np.allclose(K, geometry.cluster_momenta(a1, a2), atol=1e-15)


def test_null_walker_calls(lib):
    assert lib.dcax_walker_destroy(None) == 0
    k = ctypes.c_int32()
    assert lib.dcax_get_order(None, 0, ctypes.byref(k)) == -1
    assert lib.dcax_sweep(None, 1, None, 0, None) == -1


def test_drift_reduction_propagates_nan(tmp_path):
    """The refresh's drift reductions use max_nan from the library's device
    header: a NaN entry on either side must survive a max-reduction (IEEE fmax
    would drop it and report the NaN matrix as drift 0)."""
    import re
    import shutil
    import subprocess
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    src = open(os.path.join(ROOT, "paper_1901_01047_amd", "csrc", "dcax_dev.h")).read()
    fn = re.search(r"__host__ __device__ inline double max_nan\(double a, double b\) \{[^}]*\}", src).group(0)
    prog = tmp_path / "m.cpp"
    prog.write_text("#include <cmath>\n#include <cstdio>\n#define __host__\n#define __device__\n" + fn + """
int main() {
  const double nan = std::nan("");
  double xs[6] = {0.5, 2.0, nan, 1.0, 0.0, 3.0};
  int bad = 0;
  // a left-to-right reduction and a pairwise tree, as in the kernels
  double a = 0.0;
  for (double x : xs) a = max_nan(a, x);
  bad += !std::isnan(a);
  double t[8] = {0.5, 2.0, 1.0, nan, 0.0, 3.0, 0.25, 0.125};
  for (int o = 4; o > 0; o >>= 1)
    for (int i = 0; i < o; ++i) t[i] = max_nan(t[i], t[i + o]);
  bad += !std::isnan(t[0]);
  bad += max_nan(1.0, 2.0) != 2.0;
  bad += max_nan(2.0, 1.0) != 2.0;
  bad += !std::isnan(max_nan(nan, 1.0)) + !std::isnan(max_nan(1.0, nan));
  std::printf("%d\\n", bad);
  return bad;
}
""")
    exe = tmp_path / "m"
    subprocess.run(["g++", "-O2", str(prog), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout


def test_create_requires_an_allocator():
    """Every byte of device memory comes through the caller's allocator: a
    NULL allocator is an argument error, answered before any HIP call."""
    lib = dcax.load()
    p = dcax.make_params()
    h = ctypes.c_void_p()
    st = lib.dcax_walker_create(ctypes.byref(p), 1, None, None, ctypes.byref(h))
    assert st == -1 and h.value is None
    assert b"allocator" in lib.dcax_last_error()


@pytest.mark.parametrize("field,value", [("abi_version", 3), ("beta", 0.0), ("n_spin", 3), ("n_freq", 0),
                                         ("n_cg", 8), ("n_tau", 1), ("patch_points", 0), ("patch_points", 257),
                                         ("reserved", 1), ("mu", float("nan")), ("h", 0.3)])
def test_dca_create_rejects_bad_params(lib, field, value):
    """Argument errors of dcax_dca_create come back before any device work
    (n_cg 8 < n_freq 16; a field h != 0 with one spin block)."""
    p = dcax.make_dca_params(n_freq=16, n_cg=64, n_tau=50, patch_points=4)
    setattr(p, field, value)
    h = ctypes.c_void_p()
    al = dcax.Allocator(dcax.ALLOC_FN(lambda n, c: None), dcax.FREE_FN(lambda q, c: None), None)
    st = lib.dcax_dca_create(ctypes.byref(p), ctypes.byref(al), None, ctypes.byref(h))
    assert st == -1 and not h.value
    assert len(lib.dcax_last_error()) > 0


def test_dca_null_arguments(lib):
    assert lib.dcax_dca_coarse_grain(None, None, None, None) == -1
    assert lib.dcax_dca_g0_tables(None, None, None) == -1
    assert lib.dcax_dca_cluster_G(None, None, None, None, 1, None) == -1
    assert lib.dcax_dca_self_energy(None, None, None, None, 1.0, None, None) == -1
    assert lib.dcax_dca_iterate(None, None, 0, 1, 1.0, None, None, None) == -1
    assert lib.dcax_set_g0(None, None, 1, None, 0) == -1
    assert lib.dcax_dca_destroy(None) == 0
