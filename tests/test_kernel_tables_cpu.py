"""Every (edge slots, gene slots) shape the planner may pick has a compiled
kernel in each instantiation table of its precision: steady state and time
series, both methods, the serving step batches (FP32) and the real-n kernels
(FP64).  The tables are written out by hand in several translation units, so
a shape added to one list and missed in another would fail only when a
network that needs it is solved; this reads the sources instead."""
import pathlib
import re

CSRC = pathlib.Path(__file__).resolve().parent.parent / "paper_2503_18356_amd" / "csrc"


def planner_shapes(name):
    text = (CSRC / "rac_internal.h").read_text()
    m = re.search(r"constexpr Shape %s\[\] = \{(.*?)\};" % name, text, re.S)
    assert m, name
    return {(int(a), int(b)) for a, b in re.findall(r"\{(\d+),\s*(\d+)\}", m.group(1))}


def table_shapes(fname, macro):
    text = (CSRC / fname).read_text()
    return {(int(a), int(b)) for a, b in re.findall(r"%s\((\d+),\s*(\d+)\)" % macro, text)}


def test_fp32_tables_cover_the_planner_shapes():
    want = planner_shapes("kShapesF32")
    assert (10, 4) in want and (6, 2) in want and (7, 3) in want
    for f in ("kernels_f32_ss.hip", "kernels_f32_ts.hip", "kernels_f32_ss_tsit5.hip",
              "kernels_f32_ts_tsit5.hip", "kernels_f32_serve.hip"):
        got = table_shapes(f, "RAC_K")
        assert got == want, (f, sorted(want - got), sorted(got - want))


def test_fp64_tables_cover_the_planner_shapes():
    want = planner_shapes("kShapesF64")
    for f in ("kernels_f64_ss.hip", "kernels_f64_ts.hip", "kernels_f64_ss_tsit5.hip",
              "kernels_f64_ts_tsit5.hip"):
        got = table_shapes(f, "RAC_K")
        assert got == want, (f, sorted(want - got), sorted(got - want))
    for f in ("kernels_f64_realn.hip", "kernels_f64_realn_tsit5.hip"):
        got = {(int(a), int(b)) for a, b in re.findall(r"RAC_KR\(TS, M, (\d+), (\d+)\)", (CSRC / f).read_text())}
        assert got == want, (f, sorted(want - got), sorted(got - want))
