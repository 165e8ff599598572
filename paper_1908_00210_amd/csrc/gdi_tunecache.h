// gdi_tunecache.h -- the autotuner's persisted cache: a JSON file of launch choices
// keyed by device and problem shape. Host-only and HIP-free, so the host tests build
// it alone under the address and undefined-behaviour sanitizers.
//
// File format (written by dump, read by parse):
//   {"format": "gdi-tune-1",
//    "entries": {"<key>": {"<field>": <number>, ...}, ...}}
// Keys are opaque strings; fields are numbers (the tuning fields, plus "ms", the
// time the tuner measured). parse accepts any JSON whose top level is such an object
// and skips members it does not know.
#pragma once

#include <map>
#include <string>

namespace gdi_tunecache {

using Fields = std::map<std::string, double>;
using Table = std::map<std::string, Fields>;

// Returns 0 and fills *out (replacing entries with equal keys), or -1 with a message in
// *err when the text is not JSON of the format above (then *out is unchanged).
int parse(const std::string &text, Table *out, std::string *err);

// The JSON text of a table, one entry per line, keys in sorted order.
std::string dump(const Table &t);

// Reads a whole file; false if it cannot be opened or read.
bool read_file(const std::string &path, std::string *text);

// Writes a file through a temporary beside it and a rename, so that a concurrent
// reader sees the old or the new contents; false on any failure.
bool write_file(const std::string &path, const std::string &text);

}  // namespace gdi_tunecache
