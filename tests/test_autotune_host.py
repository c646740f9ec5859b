"""Host logic of the path tuner: the choice per size from measured times and
the table it writes (no GPU)."""

import os
import re

from paper_2312_01121_amd import autotune


def test_choice_keeps_the_previous_size_within_noise():
    m = {
        "f64/x/100": {"small": 5.0, "stream": 17.0},
        "f64/x/200": {"small": 10.1, "resident_8x0": 10.0, "stream": 18.0},    # within 2 %: keep small
        "f64/x/300": {"small": 12.0, "resident_8x0": 11.0, "stream": 18.5},    # 9 % faster: switch
        "f64/x/400": {"resident_8x0": 11.2, "resident_16x0s4": 11.1},          # keep resident_8x0
        "f64/x/500": {"resident_8x0": 12.0, "resident_16x0s4": 11.0},          # switch to four waves per row
    }
    best = autotune.choose(m)[("f64", "x")]
    assert best[100] == ("small", 0, 0, 1)
    assert best[200] == ("small", 0, 0, 1)
    assert best[300] == ("resident", 8, 0, 1)
    assert best[400] == ("resident", 8, 0, 1)
    assert best[500] == ("resident", 16, 0, 4)
    # without the tolerance every size takes its fastest
    strict = autotune.choose(m, keep_within=0.0)[("f64", "x")]
    assert strict[200] == ("resident", 8, 0, 1)
    assert strict[400] == ("resident", 16, 0, 4)


def test_parse_choice():
    assert autotune.parse_choice("stream") == ("stream", 0, 0, 1)
    assert autotune.parse_choice("resident_16x8s2") == ("resident", 16, 8, 2)
    assert autotune.parse_choice("resident_4x0") == ("resident", 4, 0, 1)


def test_committed_table_follows_its_measurements(tmp_path):
    """The committed path table is the choice rule applied to the times it
    lists."""
    text = open(autotune.PATH_HEADER).read()
    line = [ln for ln in text.splitlines() if ln.startswith("// {")][0]
    import json
    measured = json.loads(line[3:])
    out = tmp_path / "path_tune.hpp"
    autotune.write_path_header(autotune.choose(measured), measured, str(out))
    table = lambda s: re.findall(r"^    \{.*$", s, flags=re.M)  # noqa: E731
    assert table(out.read_text()) == table(text)
    assert os.path.exists(autotune.PATH_HEADER)
