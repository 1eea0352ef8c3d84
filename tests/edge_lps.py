"""Small degenerate LPs for the edge-case tests (shared by the CPU and GPU
tests; plain data, none of the solver's arithmetic)."""
import numpy as np

from paper_2512_06715_amd import ucgen


def cancelling_row():
    """x1 + x2 + 1e-6 x3 >= 1e8 with x1 <= 1e8, x2 <= 7e-9, x3 free below,
    min x3: the row sum 1e8 + 7e-9 rounds to 1e8, so the computed r of x3's
    implied lower bound is 0 while x = (1e8, 7e-9, -7e-3) is feasible; the
    optimum is -7e-3."""
    A = np.array([[1.0, 1.0, 1e-6]])
    return ucgen.dense_to_lp(A, np.array([1], np.uint8), np.array([1e8]),
                             np.array([0.0, 0.0, 1.0]), np.array([0.0, 0.0, -np.inf]),
                             np.array([1e8, 7e-9, np.inf]))


def one_by_one():
    """min x  s.t.  x >= 1,  0 <= x <= 5."""
    return ucgen.dense_to_lp(np.array([[1.0]]), np.array([1], np.uint8), np.array([1.0]),
                             np.array([1.0]), np.array([0.0]), np.array([5.0]))


def empty_row_and_columns():
    """An equality row with no entries (0 = 0), columns with no entries
    (boxed with costs of both signs) and a small coupled part."""
    A = np.array([[1.0, 2.0, 0.0, 0.0, 0.0],
                  [0.0, 0.0, 0.0, 0.0, 0.0],
                  [1.0, -1.0, 0.0, 0.0, 0.0]])
    return ucgen.dense_to_lp(A, np.array([1, 0, 0], np.uint8), np.array([2.0, 0.0, 0.5]),
                             np.array([1.0, 1.0, -2.0, 3.0, 0.0]),
                             np.array([0.0, 0.0, -1.0, 0.0, -4.0]),
                             np.array([4.0, 4.0, 2.0, 1.0, 4.0]))


def all_fixed():
    """Every variable fixed; the rows hold at the fixed point."""
    rng = np.random.default_rng(5)
    A = np.where(rng.random((6, 9)) < 0.5, rng.standard_normal((6, 9)), 0.0)
    A[:, 0] += 1.0
    xf = rng.uniform(-1, 1, 9)
    kind = np.array([0, 1, 0, 1, 1, 0], np.uint8)
    b = A @ xf - kind * 0.25
    return ucgen.dense_to_lp(A, kind, b, rng.standard_normal(9), xf, xf)


def zero_matrix():
    """No nonzeros: rows 0 >= -1 and 0 = 0; the box and the costs decide."""
    lp = ucgen.dense_to_lp(np.zeros((2, 4)), np.array([1, 0], np.uint8), np.array([-1.0, 0.0]),
                           np.array([1.0, -1.0, 0.5, -2.0]), np.array([0.0, 0.0, -1.0, -1.0]),
                           np.array([1.0, 2.0, 1.0, 3.0]))
    assert lp.row_ptr[-1] == 0
    return lp


def duplicate_rows():
    """Two identical equality rows and two identical >= rows (non-unique
    duals)."""
    A = np.array([[1.0, 1.0, 1.0], [1.0, 1.0, 1.0], [1.0, -1.0, 0.0], [1.0, -1.0, 0.0]])
    return ucgen.dense_to_lp(A, np.array([0, 0, 1, 1], np.uint8), np.array([2.0, 2.0, 0.0, 0.0]),
                             np.array([1.0, 2.0, 3.0]), np.zeros(3), np.full(3, 2.0))


def free_empty_column():
    """A free column with zero cost and no entries next to a small LP."""
    A = np.array([[1.0, 1.0, 0.0], [2.0, -1.0, 0.0]])
    return ucgen.dense_to_lp(A, np.array([1, 1], np.uint8), np.array([1.0, -1.0]),
                             np.array([2.0, 1.0, 0.0]), np.array([0.0, 0.0, -np.inf]),
                             np.array([3.0, 3.0, np.inf]))


CASES = {"one_by_one": one_by_one, "empty_row_and_columns": empty_row_and_columns,
         "all_fixed": all_fixed, "zero_matrix": zero_matrix, "duplicate_rows": duplicate_rows,
         "free_empty_column": free_empty_column}
