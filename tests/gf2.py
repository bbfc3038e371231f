"""Dense GF(2) linear algebra on Python integers, used to pin the oracle.

A row is an int whose bit j is the coefficient of column j; a right-hand side
is an r-bit int. This is textbook Gaussian elimination over arbitrary column
sets: no band, no window, no shifting - deliberately unlike the banded
insertion it checks.
"""


def lowest_bit(x: int) -> int:
    return (x & -x).bit_length() - 1


def echelon(rows, rhs):
    """Eliminate rows in the given order; pivot of a row = its lowest column.
    Returns (consistent, {pivot: (row, rhs)})."""
    piv = {}
    for row, v in zip(rows, rhs):
        while row:
            p = lowest_bit(row)
            if p not in piv:
                break
            prow, pv = piv[p]
            row ^= prow
            v ^= pv
        if row == 0:
            if v != 0:
                return False, None
            continue
        piv[lowest_bit(row)] = (row, v)
    return True, piv


def consistent(rows, rhs) -> bool:
    return echelon(rows, rhs)[0]


def solve(rows, rhs, m):
    """Solution with every non-pivot column set to 0, or None if inconsistent.

    The pivot columns (lowest column of each row of an echelon basis) depend
    only on the row space, so the solution with zero free columns is unique.
    """
    ok, piv = echelon(rows, rhs)
    if not ok:
        return None
    Z = [0] * m
    for p in sorted(piv, reverse=True):
        row, v = piv[p]
        z = v
        rest = row & ~(1 << p)
        while rest:
            q = lowest_bit(rest)
            z ^= Z[q]
            rest &= rest - 1
        Z[p] = z
    return Z


def check(rows, rhs, Z) -> bool:
    """H Z == F row by row."""
    for row, v in zip(rows, rhs):
        acc = 0
        while row:
            q = lowest_bit(row)
            acc ^= Z[q]
            row &= row - 1
        if acc != v:
            return False
    return True
