"""Run the launch-parameter autotuner on the current GPU and write the
package's default tuning file (loaded by every new context).

    python -m paper_2103_01983_amd.tune [output_path]
"""
import sys

from . import native


def main(argv):
    path = argv[1] if len(argv) > 1 else native.TUNING_PATH
    native.autotune(path)
    with open(path) as fh:
        print(fh.read(), end="")
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
