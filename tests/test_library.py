"""Host-side checks of the C-ABI library (no GPU needed)."""
import os
import re
import subprocess

import pytest

from paper_1505_03615_amd import camfe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "camfe.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(camfe_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(camfe.LIB_PATH):
        pytest.fail("libcamfe.so is not built (run __graft_entry__.build())")
    return camfe.load()


def test_every_declared_function_is_exported(lib):
    decl = declared_functions()
    assert len(decl) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", camfe.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (camfe_\w+)", out))
    missing = [f for f in decl if f not in exported]
    assert not missing, missing
    assert sorted(camfe.EXPORTS) == decl
    for f in decl:
        assert hasattr(lib, f)


def test_error_path_without_device(lib):
    import ctypes
    h = ctypes.c_void_p()
    rc = lib.camfe_ctx_create(-1, None, ctypes.byref(h))
    assert rc != 0
    assert len(lib.camfe_last_error()) > 0


def test_product_path_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_1505_03615_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "liboracle" not in txt, f


def _header_struct_fields(name):
    """Field names of `typedef struct { ... } name;` in the header, in order
    (array fields by name, pointer fields without their stars)."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + ";", src)
    assert m, name
    fields = []
    for decl in m.group(1).split(";"):
        decl = re.sub(r"\[.*?\]", "", decl).replace("*", " ").strip()
        if decl:
            first, *rest = decl.split(",")
            fields.append(first.split()[-1])
            fields.extend(r.strip() for r in rest)
    return fields


@pytest.mark.parametrize("cname,pyname", [("camfe_hier_opts", "HierOpts"), ("camfe_solve_opts", "SolveOpts"),
                                          ("camfe_solve_stats", "SolveStats"), ("camfe_train_opts", "TrainOpts"),
                                          ("camfe_eig_opts", "EigOpts"), ("camfe_eig_stats", "EigStats"),
                                          ("camfe_level_csr", "LevelCSR")])
def test_binding_structs_follow_the_header(cname, pyname):
    py = [f[0] for f in getattr(camfe, pyname)._fields_]
    assert py == _header_struct_fields(cname)


def test_training_t_per_system_is_checked_before_any_call():
    with pytest.raises(ValueError):
        camfe.camfe_smoother_train(None, [1, 2], t=[1e-3])


def test_bench_refuses_more_than_one_gpu():
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in json.loads(p.stdout.strip().splitlines()[-1])["error"]


def test_smoother_model_file_round_trip(lib, tmp_path):
    """camfe_smoother_save / camfe_smoother_load: the packed parameters, the
    BF16 flag and the sweep type survive a file; malformed files are refused."""
    import numpy as np
    rng = np.random.default_rng(3)
    params = rng.normal(size=(3, camfe.MLP_PARAMS)).astype(np.float32)
    m = camfe.camfe_model_create(params, bf16=False, sweep=camfe.SWEEP_SOR)
    path = tmp_path / "model.bin"
    camfe.camfe_smoother_save(m, path)
    raw = path.read_bytes()
    assert raw[:8] == b"CAMFESM1" and len(raw) == 8 + 16 + 4 * params.size
    assert list(np.frombuffer(raw[8:24], "<i4")) == [3, 0, 1, camfe.MLP_PARAMS]
    m2 = camfe.camfe_smoother_load(path)
    p2, bf16, sweep = camfe.camfe_model_params(m2)
    assert np.array_equal(p2, params) and bf16 is False and sweep == camfe.SWEEP_SOR
    for m_ in (m, m2):
        camfe.camfe_model_destroy(m_)
    for bad in (raw[:-4], raw + b"\0", b"CAMFESM2" + raw[8:], raw[:8] + np.array([0, 0, 1, 2081], "<i4").tobytes()
                + raw[24:], raw[:8] + np.array([3, 0, 1, 2080], "<i4").tobytes() + raw[24:]):
        path.write_bytes(bad)
        with pytest.raises(camfe.CamfeError, match="EINVAL"):
            camfe.camfe_smoother_load(path)
    with pytest.raises(camfe.CamfeError, match="EINVAL"):
        camfe.camfe_smoother_load(tmp_path / "missing.bin")
    assert lib.camfe_ctx_last_error(None) == b"null context"


class _FakeSolver:
    """Stands in for the binding in the bench's schedule choice: solve times
    and cycle counts per (smoother, sweeps at the finest depth, below)."""

    def __init__(self, table):
        self.table = table
        self.attached = []

    def camfe_smoother_attach(self, s, m):
        self.attached.append(m)

    def camfe_solve(self, s, b, t, rtol, max_iter, precision=0, smoother=0, nu_pre=2, nu_post=2, nu_coarse=0):
        secs, cyc = self.table[(smoother, nu_pre, nu_coarse)]
        if max_iter <= 4:
            return None, {"seconds": 0.0, "cycles": max_iter, "converged": False}
        return None, {"seconds": secs, "cycles": cyc, "converged": secs is not None}


def test_bench_schedule_choice_takes_each_solvers_fastest():
    """The bench's schedule choice keeps, per solver, the schedule with the
    shortest converged solve, reports a schedule that did not converge as
    null, and records every candidate's cycles."""
    import bench
    table = {}
    for sm, best in ((0, (3, 1)), (2, (2, 1)), (3, (1, 0))):
        for a, c in bench.SCHEDULES:
            table[(sm, a, c)] = (1.0 if (a, c) == best else 2.0 + a, 100 + 10 * a + c)
    table[(2, 1, 0)] = (None, 4000)     # the learned smoother does not converge with (1, 1)
    fake = _FakeSolver(table)
    out = bench.tune_schedules(fake, None, None, 1e-4, "model", [tag for tag, _ in bench.SOLVERS])
    assert out["plain_gs_fp64"]["chosen"] == [3, 1] and out["plain_gs_mixed"]["chosen"] == [3, 1]
    assert out["learned_mixed"]["chosen"] == [2, 1] and out["block_fp64"]["chosen"] == [1, 0]
    assert out["learned_mixed"]["seconds"]["1,0"] is None
    assert out["plain_gs_fp64"]["cycles"]["2,0"] == 120
    assert "model" in fake.attached and fake.attached[-1] is None
    kw = bench.schedule_kw((3, 1))
    assert kw == {"nu_pre": 3, "nu_post": 3, "nu_coarse": 1}
