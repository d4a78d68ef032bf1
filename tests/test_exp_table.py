"""The kernels' exp table (sfk_exp_table.h) holds 2^(j/512), each the
binary64 nearest the exact value: checked against a 70-digit computation
rounded once (the generator works with 60 digits), with 2^0 = 1 and
2^(1/2) the nearest binary64 to sqrt 2."""
import os
import re
from decimal import Decimal, getcontext

HERE = os.path.dirname(os.path.abspath(__file__))
HDR = os.path.join(HERE, "..", "paper_2604_21438_amd", "csrc", "sfk_exp_table.h")


def test_exp_table_matches_its_definition():
    text = open(HDR).read()
    vals = [float.fromhex(h) for h in re.findall(r"0x[0-9a-f]\.[0-9a-f]+p[+-]\d+", text)]
    assert len(vals) == 512
    getcontext().prec = 70
    ln2 = Decimal(2).ln()
    for j in range(512):
        exact = (Decimal(j) / 512 * ln2).exp()
        assert vals[j] == float(exact), j
    assert vals[0] == 1.0 and vals[256] == float(Decimal(2).sqrt())
