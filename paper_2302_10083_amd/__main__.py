"""Command line: the prime implicants of a function given by its truth table.

    python -m paper_2302_10083_amd N TABLE [--cnf] [--sliced T] [--limit K]
                                          [--rho] [--count-only]

TABLE is a file of little-endian uint32 words, bit x = f(x) with variable
x_i at bit i-1 of x (2^(N-5) words, one word for N < 5), or a hexadecimal
number prefixed with 0x for small N.  The output is the number of primes,
then the primes in increasing cube index, as strings s_1 ... s_N over
{0, 1, *} (the paper's Sec. 2 notation, s_1 leftmost), or as the indices
themselves with --rho.  --cnf lists the primes of NOT f, i.e. f's prime
clauses; --sliced T runs the sliced path with T top variables (N up to 30).
"""
import argparse
import sys

import numpy as np


def cube_string(n: int, rho: int) -> str:
    """Digits of the cube index, least significant first: 0, 1, 2 -> 0, 1, *."""
    out = []
    for _ in range(n):
        out.append("01*"[rho % 3])
        rho //= 3
    return "".join(out)


def read_table(n: int, arg: str) -> np.ndarray:
    words = 1 if n < 5 else 1 << (n - 5)
    if arg.startswith("0x"):
        v = int(arg, 16)
        if v >> (32 * words):
            raise SystemExit("the table has more than 2^%d bits" % n)
        return np.array([(v >> (32 * i)) & 0xFFFFFFFF for i in range(words)], dtype=np.uint32)
    tt = np.fromfile(arg, dtype="<u4")
    if tt.size != words:
        raise SystemExit("%s holds %d words; n = %d needs %d" % (arg, tt.size, n, words))
    return tt.astype(np.uint32)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_2302_10083_amd", description=__doc__.split("\n\n")[0])
    ap.add_argument("n", type=int, help="number of variables")
    ap.add_argument("table", help="truth-table file, or 0x... for small n")
    ap.add_argument("--cnf", action="store_true", help="primes of NOT f (f's prime clauses)")
    ap.add_argument("--sliced", type=int, default=0, metavar="T", help="sliced path with T top variables")
    ap.add_argument("--limit", type=int, default=None, metavar="K", help="print at most K primes")
    ap.add_argument("--rho", action="store_true", help="print cube indices instead of strings")
    ap.add_argument("--count-only", action="store_true", help="print the number of primes only")
    args = ap.parse_args(argv)

    from . import dqmc

    tt = read_table(args.n, args.table)
    flags = dqmc.DQMC_NEGATE if args.cnf else 0
    with dqmc.Context(0) as ctx:
        ttd = ctx.tt_to_device(tt)
        if args.sliced:
            lst, count = ctx.sliced_primes(args.n, args.sliced, ttd, list_cap=0 if args.count_only else None,
                                           flags=flags)
        elif args.count_only:
            _, lst, count = ctx.primes(args.n, ttd, list_cap=0, flags=flags)
        else:
            _, lst, count = ctx.primes(args.n, ttd, flags=flags)
        c = int(count.item())
        print(c)
        if not args.count_only:
            k = c if args.limit is None else min(c, args.limit)
            for r in lst[:k].cpu().numpy().tolist():
                print(r if args.rho else cube_string(args.n, int(r)))
    return 0


if __name__ == "__main__":
    sys.exit(main())
