"""Writes the stored expected values under tests/golden/ from the CPU oracle only.

Run from the repository root:  python tests/golden/make_golden.py
Every file it writes is checked in the test-suite against properties that do
not come from the oracle (orders found by brute force, hand-derived closed
forms), so a wrong oracle cannot silently produce a wrong fixture.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import codec, field  # noqa: E402


def main():
    with open(os.path.join(HERE, "roots.txt"), "w") as f:
        f.write("# n  r_n=3^(65536/n)  r_n^-1  n^-1   (mod 65537; root choice of Sec. II-B)\n")
        for i in range(17):
            n = 1 << i
            r = field.root(n)
            f.write(f"{n} {r} {field.inverse(r)} {field.inverse(n)}\n")
    with open(os.path.join(HERE, "worked_n4.txt"), "w") as f:
        f.write("# n=4, k=2, source s=(1, 65535): encoder output e_i = s(r_4^i) (Sec. II-B)\n")
        f.write("# by hand: r_4^2 = -1, so e = (1-2, 1-2r, 1+2, 1+2r) with r = r_4\n")
        e = codec.encode([1, 65535], 4)
        f.write(" ".join(str(int(x)) for x in e) + "\n")


if __name__ == "__main__":
    main()
