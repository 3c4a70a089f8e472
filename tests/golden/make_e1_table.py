"""Writes e1_table.txt from mpmath (50-digit arithmetic)."""
import os
import mpmath as mp

mp.mp.dps = 50
ZS = ["1e-12", "1e-3", "0.5", "1", "10", "100", "700"]
with open(os.path.join(os.path.dirname(__file__), "e1_table.txt"), "w") as f:
    f.write("# Exponential integral E1(z) = int_z^inf exp(-t)/t dt, 20 significant digits.\n")
    f.write("# Written by tests/golden/make_e1_table.py from mpmath at 50 digits (independent of both code paths).\n")
    f.write("# z  E1(z)\n")
    for z in ZS:
        f.write(f"{z} {mp.nstr(mp.e1(mp.mpf(z)), 20)}\n")
