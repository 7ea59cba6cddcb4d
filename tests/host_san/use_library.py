"""pytest plugin (test infrastructure): load the libhisv.so build named by
HISV_TEST_LIBRARY instead of the in-tree one, and report at the end of the
session which build the process mapped."""

import os

from paper_2205_06973_amd import hisv

hisv.LIB_PATH = os.environ["HISV_TEST_LIBRARY"]


def pytest_sessionfinish(session, exitstatus):
    with open("/proc/self/maps") as f:
        mapped = {line.split()[-1] for line in f if "libhisv" in line}
    print("\nmapped libhisv builds:", " ".join(sorted(mapped)))
