"""Write tests/golden/tables.json: the oracle's float32 constant tables as hex
floats, for Bz = 0.5 T.  Calls only the oracle."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def main():
    t = oracle.tables(0.5)
    doc = {"bz_tesla": 0.5,
           "note": "float32 tables of the track model, hex; rows 0..151, d = 0..17",
           "npads": [int(v) for v in oracle.npads()]}
    for k, v in t.items():
        if hasattr(v, "shape") and v.shape:
            doc[k] = [float(x).hex() for x in v]
        else:
            doc[k] = float(v).hex()
    with open(os.path.join(HERE, "tables.json"), "w") as f:
        f.write("{\n" + ",\n".join(f" {json.dumps(k)}: {json.dumps(v)}" for k, v in doc.items())
                + "\n}\n")


if __name__ == "__main__":
    main()
