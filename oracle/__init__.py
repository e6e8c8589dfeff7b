"""Reference emulator (test infrastructure only; see ``oracle/vcs_oracle.c``)."""
