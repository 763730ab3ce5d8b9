"""Measurement reports of the GPU report tests: each test prints its report
to stdout, and also writes it as JSON to $MCS_REPORT_DIR/<name> when that
variable names a directory to keep it in."""
import json
import os


def write_report(name: str, report: dict) -> None:
    out = os.environ.get("MCS_REPORT_DIR")
    if not out:
        return
    os.makedirs(out, exist_ok=True)
    with open(os.path.join(out, name), "w") as f:
        json.dump(report, f, indent=1)
