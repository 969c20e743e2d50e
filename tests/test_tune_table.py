"""CPU checks of the launch-shape table (mpsb_tune_*): entries set, read,
erased, saved and loaded; malformed text rejected without touching the
table; the default table found through MPSV_TUNING and next to the
library; the committed table well formed."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2205_11990_amd", "libmpsvlasov.so")
TABLE = os.path.join(ROOT, "paper_2205_11990_amd", "tuning_gfx950.txt")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB),
                                reason="HIP library not built (run __graft_entry__.build())")


@pytest.fixture
def B():
    from paper_2205_11990_amd import binding
    binding.lib()
    binding.tune_clear()
    yield binding
    binding.tune_clear()


def test_set_get_erase(B):
    k = (1, 300, 200, 70, 4 * 1 + 3, 0)
    assert B.tune_get(k) is None
    B.tune_set(k, 1)
    assert B.tune_get(k) == 1 and B.tune_size() == 1
    B.tune_set(k, 0)
    assert B.tune_get(k) == 0 and B.tune_size() == 1
    # another instance class is another key
    assert B.tune_get(k[:5] + (3,)) is None
    B.tune_set(k, -1)
    assert B.tune_get(k) is None and B.tune_size() == 0


@pytest.mark.parametrize("key,value", [((7, 1, 1, 1, 1, 0), 0),      # unknown knob
                                       ((1, -5, 1, 1, 1, 0), 0),     # negative key
                                       ((2, 64, 16, 32, 2, 0), 32)])  # value too large
def test_bad_entries_are_refused(B, key, value):
    with pytest.raises(B.MpsError) as e:
        B.tune_set(key, value)
    assert e.value.status == B.MPS_EINVAL
    assert B.tune_size() == 0


def test_save_load_round_trip(B, tmp_path):
    entries = {(1, 512, 512, 64, 7, 3): 1, (2, 1024, 128, 64, 2, 0): 2,
               (2, 2048, 128, 64, 3, 3): 1, (1, 65, 17, 9, 4, 1): 0}
    for k, v in entries.items():
        B.tune_set(k, v)
    p = str(tmp_path / "t.txt")
    B.tune_save(p)
    B.tune_clear()
    assert B.tune_size() == 0
    B.tune_load(p)
    assert B.tune_size() == len(entries)
    for k, v in entries.items():
        assert B.tune_get(k) == v
    # the text: a comment line, then one line of seven integers per entry
    lines = [l for l in open(p).read().splitlines() if l and not l.startswith("#")]
    assert len(lines) == len(entries)
    assert all(len(l.split()) == 7 for l in lines)


@pytest.mark.parametrize("text", ["1 2 3 4 5 6\n",            # six integers
                                  "1 2 3 4 5 6 7 8\n",        # eight
                                  "9 1 1 1 1 0 0\n",          # unknown knob
                                  "1 1 1 1 1 0 x\n",          # not an integer
                                  "1 1 1 1 1 0 40\n"])        # value out of range
def test_malformed_text_is_refused_and_table_kept(B, tmp_path, text):
    B.tune_set((1, 8, 8, 8, 4, 0), 1)
    p = tmp_path / "bad.txt"
    p.write_text("# header\n1 64 64 64 4 0 0\n" + text)
    with pytest.raises(B.MpsError) as e:
        B.tune_load(str(p))
    assert e.value.status == B.MPS_EINVAL
    assert B.tune_size() == 1 and B.tune_get((1, 8, 8, 8, 4, 0)) == 1


def test_missing_file_is_refused(B, tmp_path):
    with pytest.raises(B.MpsError):
        B.tune_load(str(tmp_path / "none.txt"))


def _size_in_fresh_process(env):
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2205_11990_amd import binding as B\n"
            "print(B.tune_size())\n" % ROOT)
    e = dict(os.environ)
    e.pop("MPSV_TUNING", None)
    e.update(env)
    out = subprocess.run([sys.executable, "-c", code], env=e, capture_output=True, text=True,
                         check=True, timeout=120)
    return int(out.stdout.strip().splitlines()[-1])


def test_default_table_from_environment(tmp_path):
    p = tmp_path / "mine.txt"
    p.write_text("# two entries\n1 300 200 70 7 0 1\n2 1024 128 64 2 3 2\n")
    assert _size_in_fresh_process({"MPSV_TUNING": str(p)}) == 2
    assert _size_in_fresh_process({"MPSV_TUNING": "none"}) == 0


def test_committed_table_is_the_default_and_well_formed(B):
    if not os.path.exists(TABLE):
        pytest.skip("no committed table")
    n = 0
    for line in open(TABLE).read().splitlines():
        if not line.strip() or line.lstrip().startswith("#"):
            continue
        f = [int(x) for x in line.split()]
        assert len(f) == 7 and f[0] in (1, 2) and 0 <= f[5] <= 3
        if f[0] == 1:
            assert f[6] in (0, 1, 2)
        else:
            assert f[6] in (1, 2, 4, 9, 10, 17, 18)
        n += 1
    assert _size_in_fresh_process({}) == n
