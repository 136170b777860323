"""Independent brute-force evaluation for tiny inputs (test infrastructure).

Written separately from epi3_oracle.c so that each can pin the other:
tables are tallied per (genotype tuple, class) in a dictionary, and K2 is
evaluated exactly as the logarithm of an integer.  Eq. 1 with J = 2 classes
is a sum over rows of ln((r+1)!) - ln(r_0!) - ln(r_1!), i.e.

    K2 = ln Q,  Q = prod_rows (r+1)! / (r_0! r_1!) = prod_rows (r+1) * C(r, r_1),

and Q is a positive integer, so the order of two combinations by K2 is the
order of their Q values, decided exactly with Python integers.
"""
from __future__ import annotations

import itertools
import math
from typing import Dict, List, Sequence, Tuple


def table_dict(geno: Sequence[Sequence[int]], pheno: Sequence[int], snps: Tuple[int, ...]
               ) -> Dict[Tuple[Tuple[int, ...], int], int]:
    counts: Dict[Tuple[Tuple[int, ...], int], int] = {}
    for s in range(len(pheno)):
        key = (tuple(int(geno[x][s]) for x in snps), int(pheno[s]))
        counts[key] = counts.get(key, 0) + 1
    return counts


def table(geno, pheno, snps: Tuple[int, ...]) -> List[List[int]]:
    """[2][3^k] table; row index is the genotype tuple read as base-3 digits
    (first SNP most significant); column 0 = controls, 1 = cases."""
    order = len(snps)
    d = table_dict(geno, pheno, snps)
    out = [[0] * (3 ** order) for _ in range(2)]
    for gt, row in zip(itertools.product(range(3), repeat=order), range(3 ** order)):
        out[0][row] = d.get((gt, 0), 0)
        out[1][row] = d.get((gt, 1), 0)
    return out


def q_value(t: List[List[int]]) -> int:
    q = 1
    for r0, r1 in zip(t[0], t[1]):
        r = r0 + r1
        q *= (r + 1) * math.comb(r, r1)
    return q


def k2_exact(t: List[List[int]]) -> float:
    """ln Q, correctly rounded to within an ulp or so by math.log on integers."""
    return math.log(q_value(t))


def scan(geno, pheno, order: int = 3):
    """Every combination of `order` SNPs: list of (Q, snps, table)."""
    M = len(geno)
    out = []
    for snps in itertools.combinations(range(M), order):
        t = table(geno, pheno, snps)
        out.append((q_value(t), snps, t))
    return out


def topk(geno, pheno, k: int, order: int = 3):
    """k best combinations under (Q, indices) ascending."""
    res = scan(geno, pheno, order)
    res.sort(key=lambda x: (x[0], x[1]))
    return res[:k]
