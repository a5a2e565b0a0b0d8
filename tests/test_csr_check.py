"""The canonical-CSR rule (the validation hsla_pattern_create applies on
the device, exported for host memory as hsla_csr_check) against a plain
definition, on Hypothesis-generated patterns: random n <= 64, densities,
empty rows; then one corruption at a time (a column out of range, an
unsorted or repeated column, a decreasing or out-of-range row pointer,
wrong end points).  Runs without a GPU."""
import numpy as np
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings  # noqa: E402
from hypothesis import strategies as st  # noqa: E402

from paper_2601_13994_amd import _lib  # noqa: E402


def first_bad_row(rp, col, n):
    """Canonical CSR by definition: row_ptr[0] = 0, row_ptr[n] = nnz, and
    for each row, in order, 0 <= row_ptr[i] <= row_ptr[i+1] <= nnz and
    columns in [0, n) strictly increasing.  Returns None, -1 (end points)
    or the first offending row."""
    nnz = len(col)
    if rp[0] != 0 or rp[n] != nnz:
        return -1
    for i in range(n):
        lo, hi = int(rp[i]), int(rp[i + 1])
        if not (0 <= lo <= hi <= nnz):
            return i
        cs = [int(c) for c in col[lo:hi]]
        if any(c < 0 or c >= n for c in cs) or any(b <= a for a, b in zip(cs, cs[1:])):
            return i
    return None


@st.composite
def canonical(draw):
    n = draw(st.integers(1, 64))
    dens = draw(st.floats(0.0, 1.0))
    rows = []
    for _ in range(n):
        k = draw(st.integers(0, max(0, int(dens * n))))
        rows.append(sorted(draw(st.sets(st.integers(0, n - 1), min_size=k, max_size=k))))
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([c for r in rows for c in r], np.int32)
    return n, rp, col


@settings(max_examples=200, deadline=None)
@given(canonical())
def test_canonical_patterns_pass(p):
    n, rp, col = p
    assert first_bad_row(rp, col, n) is None
    assert _lib.csr_check(rp, col, n) == (_lib.OK, 2**31 - 1)


CORRUPTIONS = ["col_high", "col_negative", "swap", "repeat", "rp_decrease", "rp_beyond", "end"]


@settings(max_examples=300, deadline=None)
@given(canonical(), st.sampled_from(CORRUPTIONS), st.integers(0, 10**6))
def test_corrupted_patterns_fail_at_the_first_bad_row(p, kind, pick):
    n, rp, col = p
    rp, col = rp.copy(), col.copy()
    nnz = len(col)
    full = [i for i in range(n) if rp[i + 1] > rp[i]]
    two = [i for i in range(n) if rp[i + 1] - rp[i] >= 2]
    if kind in ("col_high", "col_negative") and full:
        i = full[pick % len(full)]
        col[rp[i] + pick % (rp[i + 1] - rp[i])] = n + pick % 3 if kind == "col_high" else -1 - pick % 3
    elif kind in ("swap", "repeat") and two:
        i = two[pick % len(two)]
        k = rp[i] + pick % (rp[i + 1] - rp[i] - 1)
        if kind == "swap":
            col[k], col[k + 1] = col[k + 1], col[k]
        else:
            col[k + 1] = col[k]
    elif kind == "rp_decrease" and n >= 2 and nnz > 0:
        i = 1 + pick % (n - 1)
        rp[i] = rp[i - 1] - 1 - pick % 2 if rp[i - 1] > 0 else nnz + 1
    elif kind == "rp_beyond" and n >= 2:
        rp[1 + pick % (n - 1)] = nnz + 1 + pick % 5
    elif kind == "end":
        rp[n] = nnz + 1
    else:
        return
    want = first_bad_row(rp, col, n)
    assert want is not None
    st_, bad = _lib.csr_check(rp, col, n)
    assert st_ == _lib.ERR_INVALID_CSR and bad == want, (kind, want, bad)


def test_argument_errors():
    assert _lib.csr_check(np.zeros(1, np.int32), np.zeros(0, np.int32), -1)[0] == _lib.ERR_INVALID_ARG
    assert _lib.csr_check(np.array([0], np.int32), np.zeros(0, np.int32), 0) == (_lib.OK, 2**31 - 1)
