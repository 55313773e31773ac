"""Host-side checks of the kernel generator's plans and layouts (no GPU): every volume
row and every face trace is assigned to exactly one job, trace jobs own whole quads of
face modes (16-byte stores), the LDS area fits, and the trace layout never lets a
16-byte chunk straddle the two tangents."""
import numpy as np
import pytest

from paper_1104_4208_amd.gen import emit
from paper_1104_4208_amd.gen import tables as TB


@pytest.mark.parametrize("p", range(1, TB.P_MAX + 1))
def test_plan_partitions_rows_and_traces(p):
    t = TB.build(p)
    nw = emit.waves_for(p)
    pl = emit.plan(p, nw)
    assert len(pl["out"]) == nw and len(pl["trace"]) == nw
    rows = [b for w in pl["out"] for job in w for b in job]
    assert sorted(rows) == list(range(t.N))
    assert all(len(job) <= emit.out_rows_cap(p) for w in pl["out"] for job in w)
    traces = sorted((f, k, m) for w in pl["trace"] for f, k, ms in w for m in ms)
    assert traces == [(f, k, m) for f in range(4) for k in range(2) for m in range(t.NF)]
    for w in pl["trace"]:
        for f, k, ms in w:
            assert len(ms) <= 2 * emit.TRACE_ROWS
            for q in {m // 4 for m in ms}:  # whole quads (the last one cut at NF)
                assert set(range(4 * q, min(t.NF, 4 * q + 4))) <= set(ms)
    # output jobs are unions of whole (m, k) blocks; every stage-C2 task appears once
    blk = {r: i for i, b in enumerate(emit._blocks(t)) for r in b}
    for w in pl["out"]:
        for job in w:
            for r in job:
                assert all(q in job for q, i in blk.items() if i == blk[r])
    c2 = sorted(x for w in pl["c2"] for x in w)
    assert c2 == [(n, s) for n in range(p + 1) for s in range(2)]


@pytest.mark.parametrize("p", range(1, TB.P_MAX + 1))
def test_lds_area_fits(p):
    t = TB.build(p)
    words = emit.lds_words(p)
    assert words >= 3 * t.N * emit.LANES and words >= 8 * t.NF * emit.LANES
    assert words * 4 <= emit.LDS_BUDGET
    if p <= emit.F64_MAX_ORDER:
        assert words * 8 <= emit.LDS_BUDGET
    assert emit.groups_per_cu(p, 4) * words * 4 <= emit.LDS_BUDGET


@pytest.mark.parametrize("NF", [3, 6, 10, 15, 21, 28, 36, 45])
def test_trace_layout(NF):
    FS, ES = emit.trace_strides(NF)
    assert FS % 4 == 0 and ES == 4 * FS and FS // 2 >= NF
    NFP = FS // 2
    # value (k, m) of a face sits at k * NFP + m: every 4-chunk holds one tangent only
    pos = {(k, m): k * NFP + m for k in range(2) for m in range(NF)}
    assert len(set(pos.values())) == 2 * NF
    for (k, m), c in pos.items():
        assert c // 4 == (k * NFP + 4 * (m // 4)) // 4
        assert (c // 4) * 4 >= k * NFP and (c // 4) * 4 + 3 < (k + 1) * NFP


def test_tile_offsets_are_a_bijection():
    """Quad-interleaved tile layout: ((f FQ + j) 64 + l) 4 + i covers the tile block once."""
    NF = 28
    FS, ES = emit.trace_strides(NF)
    FQ = FS // 4
    offs = np.array([((f * FQ + j) * emit.LANES + l) * 4 + i
                     for f in range(4) for j in range(FQ) for l in range(emit.LANES) for i in range(4)])
    assert np.array_equal(np.sort(offs), np.arange(emit.LANES * ES))


def test_launcher_tables_are_indexed_by_order(tmp_path):
    """A build of a subset of the orders (here 2 and 4) puts the launcher of order p at
    index p of every table and nullptr at the orders it did not build, so the host can
    index by order and reject an order whose entry is empty."""
    import re

    emit.emit_all(str(tmp_path), [2, 4])
    src = (tmp_path / "frame.inc").read_text()
    assert "#define DGM_MAX_ORDER_F32 4" in src
    for name, stem in (("kTraceF32", "trace_p{}_f32"), ("kTraceF64", "trace_p{}_f64"), ("kPhaseF32", "phase_p{}_f32"),
                       ("kPhaseF64", "phase_p{}_f64"), ("kBatchF32", "batch_p{}_f32")):
        m = re.search(name + r"\[(\d+)\]\)\([^)]*\) = \{([^}]*)\};", src)
        assert m, name
        ents = [e.strip() for e in m.group(2).split(",")]
        assert int(m.group(1)) == 5 and len(ents) == 5, name
        for p, e in enumerate(ents):
            assert e == (f"dgm_launch_{stem.format(p)}" if p in (2, 4) else "nullptr"), (name, p, e)
    host = (tmp_path / "tables.inc").read_text()
    rows = host[host.index("kTables[5] = {"):].splitlines()[1:6]
    assert [r.strip().startswith("{0, 0,") for r in rows] == [True, True, False, True, False]
    assert rows[2].strip().startswith("{10, 6,") and rows[4].strip().startswith("{35, 15,")
