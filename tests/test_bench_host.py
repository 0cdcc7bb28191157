"""Host logic of bench.py (CPU only): the one-GPU guard and the algorithmic byte counts behind the
roofline figures."""
import ast as _ast
import os
import subprocess
import sys
from types import SimpleNamespace

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stdout


class _T:
    """Stand-in for a 1-D device tensor: numel / cpu().numpy()."""

    def __init__(self, a):
        self.a = np.asarray(a)

    def numel(self):
        return self.a.size

    def cpu(self):
        return self

    def numpy(self):
        return self.a


def test_byte_counts_follow_their_definitions():
    M, Ng, nnz = 3, 8, 10
    G = SimpleNamespace(nnz=nnz, n_work=4, tblk=_T(np.zeros(2 * 6)), n_tblk=5, fdat=_T(np.zeros(200)))
    # degrid from stored taps: taps + 4-byte columns, rowptr, perm, y, one grid read
    assert bench.degrid_bytes(G, M, Ng, 8) == 10 * 12 + 4 * 8 + 3 * 4 + 3 * 8 + 64 * 8
    # gather: transposed copy, cell offsets, block table (16 bytes per pair), y, grid written once
    assert bench.gather_bytes(G, M, Ng, 4) == 10 * 8 + 65 * 8 + 6 * 16 + 3 * 8 + 64 * 8
    # degrid from factor records: the records, their offsets, y, one grid read
    assert bench.factor_degrid_bytes(G, M, Ng) == 200 + 4 * 8 + 3 * 8 + 64 * 8
    G.tblk = None
    assert bench.gather_bytes(G, M, Ng, 4) == 10 * 8 + 65 * 8 + 3 * 8 + 64 * 8


def test_traffic_is_reported_only_for_the_profiled_source(tmp_path, monkeypatch):
    """profiled_traffic returns a figure only while the sparse-product source hashes as recorded."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    src = tmp_path / "paper_1307_3424_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "spmv.hip").write_bytes(b"kernel source")
    import hashlib
    h = hashlib.sha256(b"kernel source").hexdigest()[:16]
    (prof / "traffic_plain-256-fp32.md").write_text(f"spmv_source_sha256_16={h}\ntraffic_bytes.k_degrid=1234\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic("plain-256-fp32", "k_degrid") == 1234.0
    assert bench.profiled_traffic("plain-256-fp32", "k_gather_wave") is None
    (src / "spmv.hip").write_bytes(b"changed source")
    assert bench.profiled_traffic("plain-256-fp32", "k_degrid") is None
    # the surrogate's kernels are keyed to their own source
    (src / "surrogate.hip").write_bytes(b"network kernels")
    hs = hashlib.sha256(b"network kernels").hexdigest()[:16]
    (prof / "traffic_surrogate-2048.md").write_text(f"surrogate_source_sha256_16={hs}\ntraffic_bytes.k_sur_grid=99\n")
    assert bench.profiled_traffic("surrogate-2048", "k_sur_grid", "surrogate") == 99.0
    assert bench.profiled_traffic("surrogate-2048", "k_sur_grid") is None


# ---- a nested scope (comprehension, lambda, inner function) that reads a name its enclosing
# function binds only on a later line raises NameError when it runs; the timed GPU runs reach such
# lines only at their end, so the benchmark's and the binding's sources are checked here

_NESTED = (_ast.ListComp, _ast.SetComp, _ast.DictComp, _ast.GeneratorExp, _ast.Lambda, _ast.FunctionDef,
           _ast.AsyncFunctionDef)


def _late_free_reads(src):
    out = []
    for fn in _ast.walk(_ast.parse(src)):
        if not isinstance(fn, (_ast.FunctionDef, _ast.AsyncFunctionDef)):
            continue
        own, nested, stack = [], [], list(_ast.iter_child_nodes(fn))
        while stack:
            n = stack.pop()
            if isinstance(n, _NESTED):
                nested.append(n)
                continue
            own.append(n)
            stack.extend(_ast.iter_child_nodes(n))
        first = {}
        for n in own:
            if isinstance(n, _ast.Name) and isinstance(n.ctx, _ast.Store):
                first[n.id] = min(first.get(n.id, n.lineno), n.lineno)
        params = {a.arg for a in _ast.walk(fn.args) if isinstance(a, _ast.arg)}
        for sc in nested:
            inner = {n.id for n in _ast.walk(sc) if isinstance(n, _ast.Name) and isinstance(n.ctx, _ast.Store)}
            inner |= {a.arg for a in _ast.walk(sc) if isinstance(a, _ast.arg)}
            for n in _ast.walk(sc):
                if (isinstance(n, _ast.Name) and isinstance(n.ctx, _ast.Load) and n.id in first
                        and n.id not in inner and n.id not in params and first[n.id] > sc.lineno):
                    out.append((fn.name, n.id, n.lineno))
    return out


def test_late_free_read_check_catches_the_pattern():
    bad = "def f():\n    xs = [t + k for k in (1, 2)]\n    t = 3\n    return xs\n"
    good = "def f():\n    t = 3\n    xs = [t + k for k in (1, 2)]\n    return xs\n"
    assert _late_free_reads(bad) == [("f", "t", 2)]
    assert _late_free_reads(good) == []


def test_no_late_free_reads_in_benchmark_and_binding():
    import glob
    files = [os.path.join(ROOT, "bench.py"), os.path.join(ROOT, "__graft_entry__.py")]
    files += sorted(glob.glob(os.path.join(ROOT, "paper_1307_3424_amd", "*.py")))
    for f in files:
        assert _late_free_reads(open(f).read()) == [], f
