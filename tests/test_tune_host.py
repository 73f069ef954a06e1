"""Host tests of the tile-shape tuner and of the library's rule lookup."""
import os
import subprocess
import sys

from paper_1808_00685_amd import binding as B
from paper_1808_00685_amd import tune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_rules_ordered_and_open_ended():
    t = {}
    for mc in (16, 64):
        for nc in (512, 2048):
            # tile 2 wins only for the largest class
            t[("f32", mc, nc)] = {1: 1.0, 2: 0.5 if (mc, nc) == (64, 2048) else 2.0}
    lines = tune.rules_from_timings(t)
    rows = [tuple(int(x) for x in ln.split("\t")) for ln in lines]
    assert rows == [(B.PREC["f32"], 16, 512, 1), (B.PREC["f32"], 16, tune.OPEN, 1),
                    (B.PREC["f32"], tune.OPEN, 512, 1), (B.PREC["f32"], tune.OPEN, tune.OPEN, 2)]


def _plan_tiles_with_table(path, cases):
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1808_00685_amd import binding as B\n"
        "for prec, m, n in %r:\n"
        "    d = B.corr2d_desc_init(m=m, n1=n, prec=prec)\n"
        "    _, h = B.corr2d_plan(d)\n"
        "    print(B.corr2d_plan_get_info(h).tile)\n"
        "    B.corr2d_plan_destroy(h)\n" % (ROOT, cases))
    env = dict(os.environ, CORR2D_TUNE_TABLE=path)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr
    return [int(x) for x in out.stdout.split()]


def test_library_follows_table(tmp_path):
    p = tmp_path / "t.tsv"
    f32, split = B.PREC["f32"], B.PREC["split_bf16"]
    # f32: tile 2 up to n = 600, then tile 1; split: tile 2 everywhere;
    # a rule naming a tile the precision lacks is skipped
    p.write_text(f"# comment\n{f32}\t100\t600\t2\n{f32}\t{tune.OPEN}\t{tune.OPEN}\t1\n"
                 f"{split}\t{tune.OPEN}\t{tune.OPEN}\t1\n{split}\t{tune.OPEN}\t{tune.OPEN}\t2\n")
    got = _plan_tiles_with_table(str(p), [("f32", 16, 512), ("f32", 16, 700), ("f32", 200, 512),
                                          ("split_bf16", 16, 512), ("f64", 16, 512)])
    assert got == [2, 1, 1, 2, 1]


def test_without_table_defaults(tmp_path):
    got = _plan_tiles_with_table(str(tmp_path / "missing.tsv"),
                                 [("f32", 16, 512), ("f32", 16, 4096), ("split_bf16", 256, 16384),
                                  ("f64", 256, 16384)])
    assert got == [1, 2, 3, 1]


def test_committed_table_is_valid():
    path = tune.DEFAULT_OUT
    if not os.path.exists(path):
        return
    allowed = {B.PREC[p]: set(t) for p, t in tune.CANDIDATES.items()}
    n = 0
    for ln in open(path):
        if ln.startswith("#") or not ln.strip():
            continue
        prec, m_max, n_max, tile = (int(x) for x in ln.split())
        assert tile in allowed[prec] and m_max > 0 and n_max > 0
        n += 1
    assert n > 0
