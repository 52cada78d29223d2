"""CPU checks of the topology text reader: layout, numbering, signs and
errors, and that a parsed network goes through the library's topology call."""
import numpy as np
import pytest

from paper_2503_18356_amd import inputs
from paper_2503_18356_amd import racipe as rp


def _edges(t):
    return sorted(zip(t.src.tolist(), t.dst.tolist(), t.sign.tolist()))


def test_toggle_switch_with_header():
    t, names = inputs.parse_topo("Source Target Type\nA B 2\nB A 2\n")
    assert names == ["A", "B"] and t.n_genes == 2
    assert _edges(t) == _edges(inputs.toggle_switch())


def test_numbering_comments_blank_lines_and_self_loops():
    text = "# motif\n\nZeb1 Mir200 2\n  Mir200   Zeb1 2 \nZeb1 Zeb1 1\nSnail Zeb1 1\n"
    t, names = inputs.parse_topo(text, "emt_motif")
    assert names == ["Zeb1", "Mir200", "Snail"] and t.name == "emt_motif"
    assert _edges(t) == sorted([(0, 1, -1), (1, 0, -1), (0, 0, 1), (2, 0, 1)])
    assert t.src.dtype == np.int32 and t.sign.dtype == np.int8


def test_file_is_named_after_itself(tmp_path):
    p = tmp_path / "TS.topo"
    p.write_text("Source\tTarget\tType\nA\tB\t2\nB\tA\t2\n")
    t, names = inputs.read_topo(str(p))
    assert t.name == "TS" and names == ["A", "B"] and t.n_edges == 2


@pytest.mark.parametrize("text", [
    "",                                   # no edges
    "Source Target Type\n",               # header only
    "A B\n",                              # two fields
    "A B 2 extra\n",                      # four fields
    "A B 3\n",                            # unknown type code
    "A B 1\nC D x\n",                     # non-integer type after the first line
])
def test_rejected_texts(text):
    with pytest.raises(ValueError):
        inputs.parse_topo(text)


def test_parsed_network_through_the_library():
    t, _ = inputs.parse_topo("A B 2\nB A 2\nA A 1\nC A 1\n")
    T = rp.Topology.from_inputs(t)
    assert T.n_genes == 3 and T.n_edges == 4
    dup, _ = inputs.parse_topo("A B 1\nA B 2\n")
    with pytest.raises(rp.RacError):
        rp.Topology.from_inputs(dup)
